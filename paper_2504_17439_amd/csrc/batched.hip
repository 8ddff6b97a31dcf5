// Batched self-energy moments for many molecules: a plan built once, replayed
// as one captured hipGraph.
//
// Per molecule the path is that of gw_sigma_moments (density-response
// moments, then the two contraction stages).  In mixed precision the two
// contraction stages and the digitisation between them run as grouped,
// persistent launches over a work queue of (molecule, x chunk, tile) items
// from device job tables, so a batch of small and large molecules fills the
// chip in one launch per stage instead of one under-filled launch per
// molecule.  Jobs (x chunks of one molecule, each with its stage-1
// intermediates) are packed into waves whose intermediates fit a byte cap;
// every wave is one fold, one digitisation and one contraction launch.
// Contraction splits S per job follow a work-item target, which the optional
// autotuner picks from a candidate list by timing the whole sequence.
// The recursions (and, in FP64, the contractions) run per molecule inside the
// same graph.  The sequence is enqueued once eagerly (so that every shared
// workspace slot reaches its final size) and then captured on the handle's
// own stream; gw_batch_run replays the graph on the caller's stream.
#include "mixed_jobs.h"

#include <algorithm>
#include <cmath>
#include <vector>

struct gw_batch_s {
    gwm::Handle* h = nullptr;
    int nsys = 0, nmom_max = 0, nt = 0;
    gw_screening screening = GW_TDA;
    gw_precision prec = GW_MIXED;
    gw_opts opts{};
    bool has_opts = false;
    std::vector<gw_system> sys;

    struct Mol {
        int nmo, Ap;
        long M2, lplane, rrows, rplane;
        double* R = nullptr;
        gwm::i8* Ld = nullptr;
        int* eL = nullptr;
        gwm::i8* Rd = nullptr;
        int* eR = nullptr;
        double* part = nullptr;
        int slots = 0;  // contraction split slots (all jobs of the molecule)
    };
    std::vector<Mol> mol;

    struct Job {
        int m, x0, x1;
        long zrows;              // nt * ncol
        size_t zt_off, zl_off, zd_off, ez_off;  // element offsets in the wave buffers
        int S, slot0;
    };
    std::vector<Job> jobs;
    std::vector<std::vector<int>> waves;  // job indices per wave

    // device job tables per wave
    struct WaveTab {
        gwm::FoldJob* fold = nullptr;
        gwm::ZdigJob* zdig = nullptr;
        gwm::ContractArgs* con = nullptr;
        int njobs = 0;
        bool all64 = true;  // every contraction job of the wave has 64-row tiles
        long fold_total = 0, zdig_total = 0, con_total = 0;
    };
    std::vector<WaveTab> tabs;

    void* mem = nullptr;    // per-molecule buffers
    void* zmem = nullptr;   // wave intermediates
    void* tmem = nullptr;   // job tables
    float* Zt = nullptr;
    gwm::u16* Zl = nullptr;
    gwm::i8* Zd = nullptr;
    int* eZ = nullptr;

    // branches: the per-molecule work (recursion, digit preparation) of
    // different molecules runs on separate streams, each with its own
    // workspace, forked from and joined back to the main stream
    std::vector<gwm::Handle*> br;
    std::vector<int> mol_branch;
    std::vector<hipEvent_t> ev;  // [0] fork, [1 + b] join of branch b, [1 + nbr + i] molecule i done

    int ncu = 256;
    int split_target = 512;
    int small_tile_nmo = 0;  // jobs with nmo <= this use the 64-row contraction tile
    bool graph_ok = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace gwm {

namespace {

int tile_height(const gw_batch_s* b, int nmo) { return nmo <= b->small_tile_nmo ? 64 : 128; }
int contract_tiles(int nmo, int tm) { return mixed_upper_tiles(nmo, tm); }

// S for a job of nx orbitals x: enough contraction work items for the target
int job_split(const gw_batch_s* b, int nmo, int nx, int target, int tm) {
    const int per = contract_tiles(nmo, tm) * 2 * b->nt;
    return std::max(1, std::min({64, nx, (target + per - 1) / per}));
}

// Build (or rebuild) the contraction plan and the device job tables: the
// contraction tile of each job (64 rows for nmo <= small_nmo, else 128) and
// its splits for the work-item target.
gw_status build_tables(gw_batch_s* b, int target, int small_nmo) {
    Handle* h = b->h;
    const int nt = b->nt;
    b->small_tile_nmo = small_nmo;
    for (auto& m : b->mol) m.slots = 0;
    // every job's slots are assigned before any table is built: nsplit_total is final
    for (auto& j : b->jobs) {
        const int nmo = b->mol[j.m].nmo;
        j.S = job_split(b, nmo, j.x1 - j.x0, target, tile_height(b, nmo));
        j.slot0 = b->mol[j.m].slots;
        b->mol[j.m].slots += j.S;
    }
    for (size_t w = 0; w < b->waves.size(); ++w) {
        auto& tab = b->tabs[w];
        tab.all64 = true;
        const auto& ids = b->waves[w];
        std::vector<FoldJob> fj;
        std::vector<ZdigJob> zj;
        std::vector<ContractArgs> cj;
        long fi = 0, zi = 0, ci = 0;
        for (int id : ids) {
            const auto& j = b->jobs[id];
            const auto& m = b->mol[j.m];
            const gw_system& s = b->sys[j.m];
            const long ncol = m.M2;
            float* Zt = b->Zt + j.zt_off;
            u16* Zl = b->Zl + j.zl_off;
            i8* Zd = b->Zd + j.zd_off;
            int* eZ = b->eZ + j.ez_off;
            FoldJob f = make_fold_job(nt, m.Rd, m.eR, m.Ld, m.eL, s.eps, s.naux, m.Ap, m.nmo, s.nocc, m.rplane,
                                      m.lplane, Zt, Zl);
            f.item0 = fi;
            fi += fold_groups(f);
            fj.push_back(f);
            ZdigJob z{j.zrows, m.Ap, Zt, Zl, eZ, Zd, zi};
            zi += j.zrows;
            zj.push_back(z);
            ContractArgs a{};
            a.Ld = m.Ld; a.lplane = m.lplane; a.eL = m.eL;
            a.Zd = Zd; a.zplane = j.zrows * m.Ap; a.eZ = eZ;
            a.nmo = m.nmo; a.Ap = m.Ap; a.naux = s.naux;
            a.x0 = j.x0;
            for (int sec = 0; sec < 2; ++sec) {
                const int lo = sec == 0 ? 0 : s.nocc, hi = sec == 0 ? s.nocc : m.nmo;
                const int xs0 = std::max(j.x0, lo), xs1 = std::min(j.x1, hi);
                a.xs0[sec] = xs0;
                a.nxs[sec] = std::max(0, xs1 - xs0);
            }
            a.tm = tile_height(b, m.nmo);
            tab.all64 = tab.all64 && a.tm == 64;
            a.nt = nt; a.nsplit = j.S; a.tilesN = (m.nmo + 63) / 64; a.tiles = contract_tiles(m.nmo, a.tm);
            a.ncol = ncol;
            a.part = m.part; a.nsplit_total = m.slots; a.split_off = j.slot0;
            a.item0 = ci;
            ci += contract_groups(a);
            cj.push_back(a);
        }
        tab.njobs = (int)ids.size();
        tab.fold_total = fi;
        tab.zdig_total = zi;
        tab.con_total = ci;
        GW_HIP(h, hipMemcpy(tab.fold, fj.data(), sizeof(FoldJob) * fj.size(), hipMemcpyHostToDevice));
        GW_HIP(h, hipMemcpy(tab.zdig, zj.data(), sizeof(ZdigJob) * zj.size(), hipMemcpyHostToDevice));
        GW_HIP(h, hipMemcpy(tab.con, cj.data(), sizeof(ContractArgs) * cj.size(), hipMemcpyHostToDevice));
    }
    b->split_target = target;
    return GW_OK;
}

// Per-molecule work of molecule i on handle hb.
gw_status molecule_work(gw_batch_s* b, Handle* hb, int i) {
    const int nt = b->nt;
    const gw_opts* opts = b->has_opts ? &b->opts : nullptr;
    const gw_system& s = b->sys[i];
    auto& m = b->mol[i];
    if (b->screening == GW_TDA && b->prec == GW_MIXED)
        GW_TRY(tda_moments_mixed(hb, s.nocc, s.nvir, s.naux, b->nmom_max, s.eps, s.L, m.R));
    else if (b->screening == GW_TDA)
        GW_TRY(tda_moments_f64(hb, s.nocc, s.nvir, s.naux, b->nmom_max, s.eps, s.L, m.R, nullptr));
    else if (b->prec == GW_MIXED)
        GW_TRY(rpa_moments_mixed(hb, s.nocc, s.nvir, s.naux, b->nmom_max, s.eps, s.L, opts, m.R));
    else
        GW_TRY(rpa_moments_f64(hb, s.nocc, s.nvir, s.naux, b->nmom_max, s.eps, s.L, opts, m.R, nullptr));
    if (b->prec == GW_MIXED) GW_TRY(mixed_prep(hb, s.naux, m.nmo, nt, s.L, m.R, m.Ld, m.eL, m.Rd, m.eR));
    else
        GW_TRY(sigma_from_R_f64(hb, s.nocc, s.nvir, s.naux, b->nmom_max, s.eps, s.L, m.R, opts, s.sigma_occ,
                                s.sigma_vir));
    return GW_OK;
}

// The whole launch sequence on h->stream (forking to the branch streams).
gw_status enqueue(gw_batch_s* b) {
    Handle* h = b->h;
    const int nt = b->nt;
    if (b->prec == GW_MIXED)
        for (auto& m : b->mol) GW_TRY(fill_f64(h, m.part, (size_t)2 * nt * m.slots * m.M2, 0.0));
    if (b->br.empty()) {
        for (int i = 0; i < b->nsys; ++i) GW_TRY(molecule_work(b, h, i));
    } else {
        GW_HIP(h, hipEventRecord(b->ev[0], h->stream));
        for (auto* hb : b->br) GW_HIP(h, hipStreamWaitEvent(hb->stream, b->ev[0], 0));
        const size_t nbr = b->br.size();
        for (int i = 0; i < b->nsys; ++i) {
            Handle* hb = b->br[b->mol_branch[i]];
            gw_status st = molecule_work(b, hb, i);
            if (st != GW_OK) return set_err(h, st, hb->last_error);
            GW_HIP(h, hipEventRecord(b->ev[1 + nbr + i], hb->stream));
        }
    }
    if (b->prec != GW_MIXED) {
        for (size_t k = 0; k < b->br.size(); ++k) {
            GW_HIP(h, hipEventRecord(b->ev[1 + k], b->br[k]->stream));
            GW_HIP(h, hipStreamWaitEvent(h->stream, b->ev[1 + k], 0));
        }
        return GW_OK;
    }
    for (size_t w = 0; w < b->tabs.size(); ++w) {
        auto& tab = b->tabs[w];
        // a wave needs the per-molecule work of its own molecules only
        if (!b->br.empty()) {
            int last = -1;
            for (int id : b->waves[w]) {
                const int m = b->jobs[id].m;
                if (m == last) continue;
                last = m;
                GW_HIP(h, hipStreamWaitEvent(h->stream, b->ev[1 + b->br.size() + m], 0));
            }
        }
        {
            KTimer tm(h, "sigma_fold");
            GW_TRY(launch_fold_grouped(h, nt, tab.fold, tab.njobs, tab.fold_total, b->ncu));
            tm.stop();
        }
        {
            KTimer tm(h, "mixed_zdig");
            GW_TRY(launch_zdig_grouped(h, tab.zdig, tab.njobs, tab.zdig_total));
            tm.stop();
        }
        {
            KTimer tm(h, "sigma_contract");
            GW_TRY(launch_contract_grouped(h, tab.con, tab.njobs, tab.con_total, b->ncu, tab.all64));
            tm.stop();
        }
    }
    // every branch rejoins the main stream
    for (size_t k = 0; k < b->br.size(); ++k) {
        GW_HIP(h, hipEventRecord(b->ev[1 + k], b->br[k]->stream));
        GW_HIP(h, hipStreamWaitEvent(h->stream, b->ev[1 + k], 0));
    }
    for (int i = 0; i < b->nsys; ++i) {
        const auto& m = b->mol[i];
        const gw_system& s = b->sys[i];
        const long ps = m.M2;
        GW_TRY(reduce_splits(h, m.part, m.slots, ps, nt, m.nmo, m.nmo, m.nmo, true, 1.0, 0.0, s.sigma_occ, m.M2,
                             m.nmo));
        GW_TRY(reduce_splits(h, m.part + (long)nt * m.slots * m.M2, m.slots, ps, nt, m.nmo, m.nmo, m.nmo, true, 1.0,
                             0.0, s.sigma_vir, m.M2, m.nmo));
    }
    return GW_OK;
}

gw_status time_sequence(gw_batch_s* b, float* ms) {
    Handle* h = b->h;
    hipEvent_t e0, e1;
    GW_HIP(h, hipEventCreate(&e0));
    GW_HIP(h, hipEventCreate(&e1));
    GW_HIP(h, hipEventRecord(e0, h->stream));
    gw_status st = enqueue(b);
    GW_HIP(h, hipEventRecord(e1, h->stream));
    GW_HIP(h, hipEventSynchronize(e1));
    GW_HIP(h, hipEventElapsedTime(ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}

void release(gw_batch_s* b) {
    for (auto* hb : b->br) {
        (void)hipStreamSynchronize(hb->stream);
        for (auto& w : hb->ws)
            if (w.ptr) (void)hipFree(w.ptr);
        if (hb->own_stream) (void)hipStreamDestroy(hb->own_stream);
        delete hb;
    }
    b->br.clear();
    for (auto e : b->ev)
        if (e) (void)hipEventDestroy(e);
    b->ev.clear();
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->mem) (void)hipFree(b->mem);
    if (b->zmem) (void)hipFree(b->zmem);
    if (b->tmem) (void)hipFree(b->tmem);
    b->exec = nullptr;
    b->graph = nullptr;
    b->mem = b->zmem = b->tmem = nullptr;
}

}  // namespace

gw_status batch_create(Handle* h, int nsys, const gw_system* sys, gw_screening screening, int nmom_max,
                       gw_precision prec, const gw_opts* opts, const gw_batch_opts* bo, gw_batch* out) {
    using Job = gw_batch_s::Job;
    auto* b = new (std::nothrow) gw_batch_s();
    if (!b) return GW_ENOMEM;
    b->h = h;
    b->nsys = nsys;
    b->nmom_max = nmom_max;
    b->nt = nmom_max + 1;
    b->screening = screening;
    b->prec = prec;
    if (opts) {
        b->opts = *opts;
        b->has_opts = true;
    }
    b->sys.assign(sys, sys + nsys);
    const size_t job_bytes = (bo && bo->job_bytes) ? bo->job_bytes : ((size_t)4 << 30);
    const size_t wave_bytes = std::max(job_bytes, (bo && bo->wave_bytes) ? bo->wave_bytes : ((size_t)24 << 30));
    const bool want_graph = !(bo && bo->no_graph) && screening == GW_TDA;
    const bool autotune = bo && bo->autotune && prec == GW_MIXED;
    const int nt = b->nt;
    (void)hipDeviceGetAttribute(&b->ncu, hipDeviceAttributeMultiprocessorCount, h->device);

    // ---- per-molecule plans and jobs
    const int max_target = 2048;
    size_t bytes = 0;
    auto align = [](size_t x) { return (x + 255) & ~(size_t)255; };
    b->mol.resize(nsys);
    for (int i = 0; i < nsys; ++i) {
        auto& m = b->mol[i];
        const gw_system& s = sys[i];
        m.nmo = s.nocc + s.nvir;
        m.Ap = mixed_Ap(s.naux);
        m.M2 = (long)m.nmo * m.nmo;
        m.lplane = m.M2 * m.Ap;
        m.rrows = (long)nt * s.naux;
        m.rplane = m.rrows * m.Ap;
        if (prec == GW_MIXED && ((long)nt * s.naux * 64 >= (1L << 31) || m.M2 * 64 >= (1L << 31) || m.Ap > 4096)) {
            release(b);
            delete b;
            return set_err(h, GW_EINVAL, "batch: a molecule exceeds the mixed-precision size limits");
        }
        bytes += align(sizeof(double) * nt * (size_t)s.naux * s.naux);
        if (prec == GW_MIXED) {
            bytes += align(sizeof(i8) * MIX_ND * m.lplane) + align(sizeof(int) * (m.M2 + m.rrows)) +
                     align(sizeof(i8) * MIX_ND * m.rplane);
            // one job per molecule: stage 1 forms each symmetric (x, y) pair once
            // and writes both of its columns, so all nmo^2 columns are kept at once
            if ((long)nt * m.M2 * 64 >= (1L << 31)) {
                release(b);
                delete b;
                return set_err(h, GW_EINVAL, "batch: a molecule's nt * nmo^2 rows exceed 31-bit offsets");
            }
            Job j{};
            j.m = i;
            j.x0 = 0;
            j.x1 = m.nmo;
            j.zrows = (long)nt * m.M2;
            b->jobs.push_back(j);
            // the 128-row tile has the fewest tiles, so the most splits
            const int slots_max = job_split(b, m.nmo, m.nmo, max_target, 128);
            bytes += align(sizeof(double) * 2 * nt * (size_t)slots_max * m.M2);
            m.slots = slots_max;
        }
    }
    // ---- waves: consecutive jobs while their intermediates fit wave_bytes
    size_t zt_max = 0, zl_max = 0, zd_max = 0, ez_max = 0;
    if (prec == GW_MIXED) {
        size_t zt = 0, zl = 0, zd = 0, ez = 0, used = 0;
        std::vector<int> cur;
        for (size_t k = 0; k < b->jobs.size(); ++k) {
            auto& j = b->jobs[k];
            const size_t e = (size_t)j.zrows * b->mol[j.m].Ap;
            const size_t jb = e * (sizeof(float) + sizeof(u16) + MIX_ND * sizeof(i8)) + sizeof(int) * j.zrows;
            if (!cur.empty() && used + jb > wave_bytes) {
                b->waves.push_back(cur);
                cur.clear();
                zt = zl = zd = ez = used = 0;
            }
            j.zt_off = zt;
            j.zl_off = zl;
            j.zd_off = zd;
            j.ez_off = ez;
            zt += (e + 63) & ~(size_t)63;
            zl += (e + 127) & ~(size_t)127;
            zd += MIX_ND * ((e + 127) & ~(size_t)127);
            ez += (j.zrows + 63) & ~(size_t)63;
            used += jb;
            zt_max = std::max(zt_max, zt);
            zl_max = std::max(zl_max, zl);
            zd_max = std::max(zd_max, zd);
            ez_max = std::max(ez_max, ez);
            cur.push_back((int)k);
        }
        if (!cur.empty()) b->waves.push_back(cur);
    }
    // ---- allocation
    if (hipMalloc(&b->mem, std::max<size_t>(bytes, 256)) != hipSuccess) {
        (void)hipGetLastError();
        release(b);
        delete b;
        return set_err(h, GW_ENOMEM, "batch: device allocation failed (" + std::to_string(bytes) + " bytes)");
    }
    {
        char* p = (char*)b->mem;
        for (int i = 0; i < nsys; ++i) {
            auto& m = b->mol[i];
            const gw_system& s = sys[i];
            m.R = (double*)p;
            p += align(sizeof(double) * nt * (size_t)s.naux * s.naux);
            if (prec != GW_MIXED) continue;
            m.Ld = (i8*)p;
            p += align(sizeof(i8) * MIX_ND * m.lplane);
            m.eL = (int*)p;
            m.eR = m.eL + m.M2;
            p += align(sizeof(int) * (m.M2 + m.rrows));
            m.Rd = (i8*)p;
            p += align(sizeof(i8) * MIX_ND * m.rplane);
            m.part = (double*)p;
            p += align(sizeof(double) * 2 * nt * (size_t)m.slots * m.M2);
        }
    }
    if (prec == GW_MIXED) {
        const size_t zb = sizeof(float) * zt_max + sizeof(u16) * zl_max + sizeof(i8) * zd_max + sizeof(int) * ez_max + 4096;
        const size_t nw = b->waves.size(), nj = b->jobs.size();
        const size_t tb = (sizeof(FoldJob) + sizeof(ZdigJob) + sizeof(ContractArgs)) * nj + 3 * 256 * nw;
        if (hipMalloc(&b->zmem, zb) != hipSuccess || hipMalloc(&b->tmem, tb) != hipSuccess) {
            (void)hipGetLastError();
            release(b);
            delete b;
            return set_err(h, GW_ENOMEM, "batch: wave buffer allocation failed");
        }
        char* p = (char*)b->zmem;
        b->Zt = (float*)p;
        p += align(sizeof(float) * zt_max);
        b->Zl = (u16*)p;
        p += align(sizeof(u16) * zl_max);
        b->Zd = (i8*)p;
        p += align(sizeof(i8) * zd_max);
        b->eZ = (int*)p;
        char* t = (char*)b->tmem;
        b->tabs.resize(nw);
        for (size_t w = 0; w < nw; ++w) {
            const size_t n = b->waves[w].size();
            b->tabs[w].fold = (FoldJob*)t;
            t += align(sizeof(FoldJob) * n);
            b->tabs[w].zdig = (ZdigJob*)t;
            t += align(sizeof(ZdigJob) * n);
            b->tabs[w].con = (ContractArgs*)t;
            t += align(sizeof(ContractArgs) * n);
        }
    }

    // ---- branches (TDA: the per-molecule path uses no library handle); molecules
    // assigned largest first to the least loaded branch by cost ~ nmo^4.  A
    // TDA batch always has at least one branch with its own workspace: the
    // captured graph then references batch-owned memory only, never the
    // caller handle's workspace (which a later, larger call may reallocate).
    const int nbr = screening == GW_TDA ? std::min((bo && bo->branches > 0) ? bo->branches : 4, nsys) : 0;
    if (nbr >= 1) {
        b->ev.assign(1 + nbr + nsys, nullptr);
        for (auto& e : b->ev)
            if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
                (void)hipGetLastError();
                release(b);
                delete b;
                return set_err(h, GW_EHIP, "batch: event creation failed");
            }
        for (int k = 0; k < nbr; ++k) {
            auto* hb = new (std::nothrow) Handle();
            if (!hb || hipStreamCreateWithFlags(&hb->own_stream, hipStreamNonBlocking) != hipSuccess) {
                (void)hipGetLastError();
                delete hb;
                release(b);
                delete b;
                return set_err(h, GW_EHIP, "batch: branch stream creation failed");
            }
            hb->device = h->device;
            hb->stream = hb->own_stream;
            hb->ws.resize(WS_COUNT);
            b->br.push_back(hb);
        }
        std::vector<int> order(nsys);
        for (int i = 0; i < nsys; ++i) order[i] = i;
        auto cost = [&](int i) { return std::pow((double)b->mol[i].nmo, 4.0); };
        std::sort(order.begin(), order.end(), [&](int x, int y) { return cost(x) > cost(y); });
        std::vector<double> load(nbr, 0.0);
        b->mol_branch.assign(nsys, 0);
        for (int i : order) {
            const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
            b->mol_branch[i] = k;
            load[k] += cost(i);
        }
    }

    // ---- contraction split plan (optionally autotuned), eager warm-up
    const bool timing = h->timing;
    gw_status st = GW_OK;
    const int small0 = (bo && bo->small_tile_nmo > 0) ? bo->small_tile_nmo : 0;
    if (prec == GW_MIXED) st = build_tables(b, (bo && bo->split_target > 0) ? bo->split_target : 512, small0);
    if (st == GW_OK) st = enqueue(b);  // grows the shared workspace to its final size
    if (st == GW_OK) {
        hipError_t e = hipStreamSynchronize(h->stream);
        if (e != hipSuccess) st = set_err(h, GW_EHIP, std::string("batch warm-up: ") + hipGetErrorString(e));
    }
    if (st == GW_OK && autotune) {
        // coordinate search: the split target with 128-row tiles only, then
        // the largest nmo that takes the 64-row contraction tile (1 << 20:
        // every molecule, which also gives the launch two work groups per CU)
        h->timing = false;
        int best = b->split_target, best_small = 0;
        float best_ms = 1e30f;
        for (int target : {256, 512, 1024, 2048}) {
            st = build_tables(b, target, 0);
            float ms = 0.f;
            if (st == GW_OK) st = time_sequence(b, &ms);
            if (st != GW_OK) break;
            if (ms < best_ms) {
                best_ms = ms;
                best = target;
            }
        }
        for (int small : {100, 150, 200, 1 << 20}) {
            if (st != GW_OK) break;
            st = build_tables(b, best, small);
            float ms = 0.f;
            if (st == GW_OK) st = time_sequence(b, &ms);
            if (st != GW_OK) break;
            if (ms < best_ms) {
                best_ms = ms;
                best_small = small;
            }
        }
        if (st == GW_OK) st = build_tables(b, best, best_small);
        h->timing = timing;
    }
    // ---- capture
    if (st == GW_OK && want_graph) {
        hipStream_t caller = h->stream;
        h->stream = h->own_stream;
        rocblas_set_stream(h->blas, h->stream);
        h->timing = false;
        hipError_t e = hipStreamBeginCapture(h->stream, hipStreamCaptureModeRelaxed);
        gw_status es = GW_OK;
        if (e == hipSuccess) {
            es = enqueue(b);
            hipGraph_t g = nullptr;
            e = hipStreamEndCapture(h->stream, &g);
            if (e == hipSuccess && es == GW_OK) {
                b->graph = g;
                e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
                b->graph_ok = (e == hipSuccess);
            } else if (g) {
                (void)hipGraphDestroy(g);
            }
        }
        (void)hipGetLastError();
        h->timing = timing;
        h->stream = caller;
        rocblas_set_stream(h->blas, h->stream);
        if (!b->graph_ok) st = set_err(h, GW_EHIP, "batch: graph capture failed");
    }
    if (st != GW_OK) {
        release(b);
        delete b;
        return st;
    }
    *out = b;
    return GW_OK;
}

gw_status batch_run(gw_batch b) {
    Handle* h = b->h;
    if (b->graph_ok) {
        GW_HIP(h, hipGraphLaunch(b->exec, h->stream));
        return GW_OK;
    }
    return enqueue(b);
}

gw_status batch_info(gw_batch b, int* njobs, int* nwaves, int* graph, int* split_target, int* small_tile_nmo) {
    if (small_tile_nmo) *small_tile_nmo = b->small_tile_nmo;
    if (njobs) *njobs = (int)b->jobs.size();
    if (nwaves) *nwaves = (int)b->waves.size();
    if (graph) *graph = b->graph_ok ? 1 : 0;
    if (split_target) *split_target = b->split_target;
    return GW_OK;
}

void batch_destroy(gw_batch b) {
    if (!b) return;
    (void)hipStreamSynchronize(b->h->stream);
    release(b);
    delete b;
}

}  // namespace gwm
