// ensemble.hip -- batched advection of an ensemble of uneven LES members.
//
// Every member advances with the mixed-precision step (FP32 source terms from
// the FP64 state, FP64 accumulation; the single-precision advection of
// Sec. 4.1).  One persistent launch per step takes (member, tile) work items
// from a list sorted by decreasing cost through an atomic cursor, whatever
// the member's column height (a member of up to 64 levels runs the one-chunk
// march, a taller one the two-chunk march, both compiled into the kernel);
// N steps are captured once into a hipGraph and replayed with one
// hipGraphLaunch.  The segment length and the persistent grid size are chosen
// by timing candidates on the plan's own members (cached in a small JSON file
// keyed by device, precision and scalar count).  With budgets attached, every
// work item also leaves one row of FP64 budget partials and a small pass sums
// each member's rows in a fixed order (the checks of every step, Sec. 3.1).
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "march.hpp"

namespace monc {

namespace {

constexpr int ENS_WAVES = march_waves<double, float>();  // FP64 state held in registers

struct EnsMember {
    AdvArgs a[2];  // a[p]: reads state[p], writes state[1-p]
    int ti;        // planes per segment
    int njt;       // tiles along y
    int nch;       // 64-level chunks per column (1 or 2)
};

template <int NS>
constexpr size_t ens_lds_bytes() {
    return std::max(march_lds_bytes<double, float, NS, 1>(), march_lds_bytes<double, float, NS, 2>());
}

// Persistent step of every member.  cursor[0] hands out work items, cursor[1]
// counts the workgroups that are done: the last one resets both, so the next
// launch (eager, timed or replayed from a graph) starts from zero.  Every
// workgroup leaves the loop once the cursor has passed the list, so all of
// them finish; the results do not depend on which workgroup takes an item.
template <int NS, bool BUD>
__global__ void __launch_bounds__(ENS_WAVES * 64) __attribute__((amdgpu_waves_per_eu(2)))
    ensemble_step(const EnsMember* __restrict__ mem, const int4* __restrict__ items, int nitems,
                  int parity, double* __restrict__ partials, int* __restrict__ cursor) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int next;
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(cursor, 1);
        __syncthreads();
        const int it = next;
        __syncthreads();  // every thread has read `next` before it is written again
        if (it >= nitems) break;
        const int4 w = items[it];
        const EnsMember* M = mem + w.x;
        TileJob t;
        t.s0 = 0;
        t.ti = M->ti;
        t.jt = w.y;
        t.seg = w.z;
        t.partial_row = BUD ? partials + (size_t)it * NB : nullptr;
        t.first_pass = 1;
        if (M->nch == 1)
            march_tile<double, float, STEP, true, NS, BUD, 1, 0>(M->a[parity], t, smem_raw);
        else
            march_tile<double, float, STEP, true, NS, BUD, 2, 0>(M->a[parity], t, smem_raw);
        __syncthreads();  // the LDS is reused by the next item
    }
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(cursor + 1, 1) == (int)gridDim.x - 1) {
            atomicExch(cursor, 0);
            atomicExch(cursor + 1, 0);
        }
    }
}

// Budgets of every member from its items' partial rows: one workgroup per
// member, lane q sums entry q over the member's rows in list order (so the
// result is repeatable bit for bit).
__global__ void __launch_bounds__(64) ensemble_budget_final(const double* __restrict__ partials,
                                                            const int* __restrict__ rowoff,
                                                            const int* __restrict__ rows,
                                                            double* __restrict__ out) {
    const int m = blockIdx.x, q = threadIdx.x;
    if (q >= NB) return;
    const int op = bud_op(q);
    double v = bud_ident(op);
    for (int r = rowoff[m]; r < rowoff[m + 1]; r++)
        v = bud_comb(v, partials[(size_t)rows[r] * NB + q], op);
    out[(size_t)m * NB + q] = v;
}

template <int NS, bool BUD>
hipError_t set_attr_one() {
    return hipFuncSetAttribute((const void*)ensemble_step<NS, BUD>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)ens_lds_bytes<NS>());
}

template <bool BUD>
hipError_t set_attrs_bud() {
    hipError_t e = set_attr_one<0, BUD>();
    if (e == hipSuccess) e = set_attr_one<1, BUD>();
    if (e == hipSuccess) e = set_attr_one<2, BUD>();
    if (e == hipSuccess) e = set_attr_one<3, BUD>();
    return e;
}

hipError_t set_attrs() {
    hipError_t e = set_attrs_bud<false>();
    if (e == hipSuccess) e = set_attrs_bud<true>();
    return e;
}

template <int NS, bool BUD>
hipError_t launch_ns(const EnsMember* mem, const int4* items, int nitems, int grid, int parity,
                     double* partials, int* cursor, hipStream_t s) {
    ensemble_step<NS, BUD><<<grid, ENS_WAVES * 64, ens_lds_bytes<NS>(), s>>>(
        mem, items, nitems, parity, partials, cursor);
    return hipGetLastError();
}

// partials: the first budget row, or nullptr (no budgets)
hipError_t launch_any(int ns, const EnsMember* mem, const int4* items, int nitems, int grid,
                      int parity, double* partials, int* cursor, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    if (partials) {
        switch (ns) {
            case 0: return launch_ns<0, true>(mem, items, nitems, grid, parity, partials, cursor, s);
            case 1: return launch_ns<1, true>(mem, items, nitems, grid, parity, partials, cursor, s);
            case 2: return launch_ns<2, true>(mem, items, nitems, grid, parity, partials, cursor, s);
            case 3: return launch_ns<3, true>(mem, items, nitems, grid, parity, partials, cursor, s);
        }
    } else {
        switch (ns) {
            case 0: return launch_ns<0, false>(mem, items, nitems, grid, parity, nullptr, cursor, s);
            case 1: return launch_ns<1, false>(mem, items, nitems, grid, parity, nullptr, cursor, s);
            case 2: return launch_ns<2, false>(mem, items, nitems, grid, parity, nullptr, cursor, s);
            case 3: return launch_ns<3, false>(mem, items, nitems, grid, parity, nullptr, cursor, s);
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace

// ---------------------------------------------------------------------------
// The plan
// ---------------------------------------------------------------------------
struct EnsemblePlan {
    int n = 0, nscal = 0;
    std::vector<monc_member> members;
    std::vector<EnsMember> hmem;
    EnsMember* d_mem = nullptr;
    int4* d_items = nullptr;
    int nitems = 0;
    int nclass[2] = {0, 0};  // items of one-chunk and two-chunk members
    int grid = 0;
    int ti = 32;
    int* d_cursor = nullptr;  // [2]: work cursor, finished workgroups
    hipStream_t cap = nullptr;
    hipGraphExec_t exec[2] = {nullptr, nullptr};  // by starting parity
    int exec_steps[2] = {0, 0};
    int parity = 0;
    std::vector<int4> hitems;  // the uploaded work list (host copy)
    // budgets (attached by the caller): slots of n x NB doubles, one per step
    // of a run; one partial row per work item and each member's row list (CSR)
    double* budgets = nullptr;
    int nslots = 0;
    double* d_partials = nullptr;
    int* d_rowoff = nullptr;
    int* d_rows = nullptr;
};

namespace {

int tj_of(int nch) { return ENS_WAVES / nch; }

// The work list for a segment length: every (member, tile) item, sorted by
// decreasing cost (planes x levels x columns), so that the workgroups taking
// items in order from the cursor finish close together.
std::vector<int4> build_items(const EnsemblePlan& P, int ti) {
    std::vector<int4> items;
    for (int m = 0; m < P.n; m++) {
        const monc_member& M = P.members[m];
        const int nch = M.nz <= 64 ? 1 : 2;
        const int tj = tj_of(nch);
        const int njt = (M.ny + tj - 1) / tj;
        const int nseg = (M.nx + ti - 1) / ti;
        for (int s = 0; s < nseg; s++) {
            const int planes = std::min(ti, M.nx - s * ti);
            for (int t = 0; t < njt; t++) items.push_back(make_int4(m, t, s, planes * tj * M.nz));
        }
    }
    std::stable_sort(items.begin(), items.end(),
                     [](const int4& a, const int4& b) { return a.w > b.w; });
    return items;
}

hipError_t upload_items(EnsemblePlan& P, int ti) {
    hipError_t e0 = hipStreamSynchronize(P.cap);  // the old list may still be in use
    if (e0 != hipSuccess) return e0;
    std::vector<int4> items = build_items(P, ti);
    if (P.d_items) {
        const hipError_t ef = hipFree(P.d_items);
        P.d_items = nullptr;
        if (ef != hipSuccess) return ef;
    }
    P.nitems = (int)items.size();
    P.nclass[0] = P.nclass[1] = 0;
    for (const int4& it : items) P.nclass[P.members[it.x].nz <= 64 ? 0 : 1]++;
    P.hitems = items;
    P.ti = ti;
    for (int m = 0; m < P.n; m++) P.hmem[m].ti = ti;
    if (items.empty()) return hipSuccess;
    hipError_t e = hipMalloc(&P.d_items, items.size() * sizeof(int4));
    if (e != hipSuccess) return e;
    return hipMemcpy(P.d_items, items.data(), items.size() * sizeof(int4), hipMemcpyHostToDevice);
}

hipError_t upload_members(EnsemblePlan& P) {
    return hipMemcpy(P.d_mem, P.hmem.data(), P.hmem.size() * sizeof(EnsMember),
                     hipMemcpyHostToDevice);
}

// One step of every member; with budgets attached, the budgets of the step's
// input state go to slot `slot`.
hipError_t launch_step(EnsemblePlan& P, int parity, int slot, hipStream_t s) {
    const bool bud = P.budgets != nullptr;
    hipError_t e = launch_any(P.nscal, P.d_mem, P.d_items, P.nitems, P.grid, parity,
                              bud ? P.d_partials : nullptr, P.d_cursor, s);
    if (e != hipSuccess) return e;
    if (bud) {
        ensemble_budget_final<<<P.n, 64, 0, s>>>(P.d_partials, P.d_rowoff, P.d_rows,
                                                 P.budgets + (size_t)slot * P.n * NB);
        return hipGetLastError();
    }
    return hipSuccess;
}

// Row lists of the members from the current work list: member m's rows are
// the indices of its items, in list order.
hipError_t build_budget_rows(EnsemblePlan& P) {
    std::vector<std::vector<int>> per(P.n);
    for (int it = 0; it < P.nitems; it++) per[P.hitems[it].x].push_back(it);
    std::vector<int> off(P.n + 1, 0), rows;
    for (int m = 0; m < P.n; m++) {
        off[m + 1] = off[m] + (int)per[m].size();
        rows.insert(rows.end(), per[m].begin(), per[m].end());
    }
    hipError_t e = hipMalloc(&P.d_partials, std::max<size_t>(P.nitems, 1) * NB * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&P.d_rowoff, off.size() * sizeof(int));
    if (e == hipSuccess) e = hipMalloc(&P.d_rows, std::max<size_t>(rows.size(), 1) * sizeof(int));
    if (e == hipSuccess)
        e = hipMemcpy(P.d_rowoff, off.data(), off.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess && !rows.empty())
        e = hipMemcpy(P.d_rows, rows.data(), rows.size() * sizeof(int), hipMemcpyHostToDevice);
    return e;
}

hipError_t free_budget_rows(EnsemblePlan& P) {
    hipError_t e = hipSuccess;
    void* bufs[3] = {P.d_partials, P.d_rowoff, P.d_rows};
    for (void* b : bufs) {
        if (!b) continue;
        const hipError_t ef = hipFree(b);
        if (e == hipSuccess) e = ef;
    }
    P.d_partials = nullptr;
    P.d_rowoff = nullptr;
    P.d_rows = nullptr;
    return e;
}

// --- tiny JSON cache: {"key": [ti, grid], ...} -------------------------------
std::string cache_key(int nscal) {
    hipDeviceProp_t prop;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return "unknown-device:" + std::to_string(nscal);
    char buf[256];
    snprintf(buf, sizeof buf, "%s|fp32-tend-fp64-state|nscal%d", prop.gcnArchName, nscal);
    return buf;
}

bool cache_read(const char* path, const std::string& key, int* ti, int* grid) {
    if (!path) return false;
    FILE* f = fopen(path, "r");
    if (!f) return false;
    std::string text;
    char buf[4096];
    size_t r;
    while ((r = fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, r);
    fclose(f);
    const std::string pat = "\"" + key + "\": [";
    const size_t p = text.find(pat);
    if (p == std::string::npos) return false;
    return sscanf(text.c_str() + p + pat.size(), "%d, %d", ti, grid) == 2;
}

void cache_write(const char* path, const std::string& key, int ti, int grid) {
    if (!path) return;
    std::vector<std::string> lines;
    FILE* f = fopen(path, "r");
    if (f) {
        char buf[1024];
        while (fgets(buf, sizeof buf, f)) {
            std::string l(buf);
            if (l.find("\": [") != std::string::npos && l.find("\"" + key + "\"") == std::string::npos) {
                while (!l.empty() && (l.back() == '\n' || l.back() == ',')) l.pop_back();
                lines.push_back(l);
            }
        }
        fclose(f);
    }
    char ent[512];
    snprintf(ent, sizeof ent, "  \"%s\": [%d, %d]", key.c_str(), ti, grid);
    lines.push_back(ent);
    f = fopen(path, "w");
    if (!f) return;
    fprintf(f, "{\n");
    for (size_t i = 0; i < lines.size(); i++)
        fprintf(f, "%s%s\n", lines[i].c_str(), i + 1 < lines.size() ? "," : "");
    fprintf(f, "}\n");
    fclose(f);
}

// Time one step (average of reps) for the current list and grid.  Timing
// writes only the members' "next" buffers.
float time_step(EnsemblePlan& P, int reps) {
    hipEvent_t a, b;
    hipEventCreate(&a);
    hipEventCreate(&b);
    launch_any(P.nscal, P.d_mem, P.d_items, P.nitems, P.grid, P.parity, nullptr, P.d_cursor, P.cap);
    hipEventRecord(a, P.cap);
    for (int r = 0; r < reps; r++)
        launch_any(P.nscal, P.d_mem, P.d_items, P.nitems, P.grid, P.parity, nullptr, P.d_cursor,
                   P.cap);
    hipEventRecord(b, P.cap);
    hipEventSynchronize(b);
    float ms = 0;
    hipEventElapsedTime(&ms, a, b);
    hipEventDestroy(a);
    hipEventDestroy(b);
    return ms / reps;
}

int num_cus() {
    int dev = 0, cus = 256;
    hipGetDevice(&dev);
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    return cus;
}

// The autotuner: segment length x persistent grid size, timed on the plan's
// own members.  Grids larger than the work list are clipped.
hipError_t tune(EnsemblePlan& P, const char* cache, bool do_tune) {
    const int cus = num_cus();
    int best_ti = 32, best_grid = cus;
    const std::string key = cache_key(P.nscal);
    const bool have = cache_read(cache, key, &best_ti, &best_grid);
    if (!have && do_tune) {
        float best = 1e30f;
        const int tis[] = {16, 32, 64, 128};
        const int grids[] = {cus, 2 * cus, 4 * cus};
        for (int ti : tis) {
            hipError_t e = upload_items(P, ti);
            if (e != hipSuccess) return e;
            e = upload_members(P);
            if (e != hipSuccess) return e;
            if (P.nitems == 0) return hipSuccess;
            for (int g : grids) {
                P.grid = std::min(g, P.nitems);
                const float ms = time_step(P, 3);
                if (ms < best) {
                    best = ms;
                    best_ti = ti;
                    best_grid = g;
                }
            }
        }
        cache_write(cache, key, best_ti, best_grid);
    }
    hipError_t e = upload_items(P, best_ti);
    if (e != hipSuccess) return e;
    P.grid = std::max(1, std::min(best_grid, P.nitems));
    return upload_members(P);
}

}  // namespace

int ensemble_create(const monc_member* members, int n, int nscal, const char* tune_cache,
                    int do_tune, EnsemblePlan** out, std::string* err) {
    EnsemblePlan* P = new EnsemblePlan();
    P->n = n;
    P->nscal = nscal;
    P->members.assign(members, members + n);
    P->hmem.resize(n);
    for (int m = 0; m < n; m++) {
        const monc_member& M = members[m];
        for (int p = 0; p < 2; p++) {
            AdvArgs& a = P->hmem[m].a[p];
            for (int f = 0; f < 3 + MAXS; f++) {
                a.in[f] = nullptr;
                a.out[f] = nullptr;
            }
            for (int f = 0; f < 3 + nscal; f++) {
                a.in[f] = M.state[p][f];
                a.out[f] = M.state[1 - p][f];
            }
            for (int s = 0; s < MAXS; s++) a.phi0[s] = s < nscal ? M.phi0[s] : 0.0;
            a.nscal = nscal;
            a.nx = M.nx;
            a.ny = M.ny;
            a.nz = M.nz;
            a.dx = M.dx;
            a.dy = M.dy;
            a.dt = M.dt;
            a.rdz = M.rdz;
            a.rho = M.rho;
            a.rhon = M.rhon;
            a.partials = nullptr;
            a.dyn = 0;
            a.fcor = a.ug = a.vg = a.gth = a.th0 = 0.0;
            a.spw = 0;
            a.work = 1;
        }
        const int nch = M.nz <= 64 ? 1 : 2;
        P->hmem[m].nch = nch;
        P->hmem[m].njt = (M.ny + tj_of(nch) - 1) / tj_of(nch);
        P->hmem[m].ti = 32;
    }
    hipError_t e = set_attrs();
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&P->cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipMalloc(&P->d_mem, sizeof(EnsMember) * n);
    if (e == hipSuccess) e = hipMalloc(&P->d_cursor, 2 * sizeof(int));
    if (e == hipSuccess) e = hipMemset(P->d_cursor, 0, 2 * sizeof(int));
    if (e == hipSuccess) e = tune(*P, tune_cache, do_tune != 0);
    if (e == hipSuccess) e = hipStreamSynchronize(P->cap);
    if (e != hipSuccess) {
        *err = hipGetErrorString(e);
        ensemble_destroy(P);
        return MONC_EHIP;
    }
    *out = P;
    return MONC_OK;
}

int ensemble_set_budgets(EnsemblePlan* P, double* budgets, int nslots, std::string* err) {
    hipError_t e = hipStreamSynchronize(P->cap);
    if (e == hipSuccess) e = hipDeviceSynchronize();  // captured graphs may still run
    for (int c = 0; c < 2; c++) {
        if (P->exec[c]) hipGraphExecDestroy(P->exec[c]);
        P->exec[c] = nullptr;
        P->exec_steps[c] = 0;
    }
    if (e == hipSuccess) e = free_budget_rows(*P);
    P->budgets = nullptr;
    P->nslots = 0;
    if (e == hipSuccess && budgets) {
        e = build_budget_rows(*P);
        if (e == hipSuccess) {
            P->budgets = budgets;
            P->nslots = nslots;
        } else {
            free_budget_rows(*P);
        }
    }
    if (e != hipSuccess) {
        *err = hipGetErrorString(e);
        return MONC_EHIP;
    }
    return MONC_OK;
}

int ensemble_budget_slots(const EnsemblePlan* P) { return P->budgets ? P->nslots : -1; }

int ensemble_step_eager(EnsemblePlan* P, hipStream_t s, std::string* err) {
    hipError_t e = launch_step(*P, P->parity, 0, s);
    if (e != hipSuccess) {
        *err = hipGetErrorString(e);
        return MONC_EHIP;
    }
    P->parity ^= 1;
    return MONC_OK;
}

int ensemble_run(EnsemblePlan* P, int nsteps, hipStream_t s, std::string* err) {
    const int p0 = P->parity;
    if (!P->exec[p0] || P->exec_steps[p0] != nsteps) {
        if (P->exec[p0]) {
            hipGraphExecDestroy(P->exec[p0]);
            P->exec[p0] = nullptr;
        }
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamBeginCapture(P->cap, hipStreamCaptureModeThreadLocal);
        for (int k = 0; k < nsteps && e == hipSuccess; k++)
            e = launch_step(*P, p0 ^ (k & 1), k, P->cap);
        hipError_t e2 = hipStreamEndCapture(P->cap, &g);
        if (e == hipSuccess) e = e2;
        if (e == hipSuccess) e = hipGraphInstantiate(&P->exec[p0], g, nullptr, nullptr, 0);
        if (g) hipGraphDestroy(g);
        if (e != hipSuccess) {
            *err = std::string("graph capture: ") + hipGetErrorString(e);
            P->exec[p0] = nullptr;
            return MONC_EHIP;
        }
        P->exec_steps[p0] = nsteps;
    }
    hipError_t e = hipGraphLaunch(P->exec[p0], s);
    if (e != hipSuccess) {
        *err = hipGetErrorString(e);
        return MONC_EHIP;
    }
    P->parity ^= (nsteps & 1);
    return MONC_OK;
}

// ti, grid, nitems: [2] each; the single list's segment length and grid in
// both entries, the items of one-chunk and two-chunk members in nitems.
void ensemble_info(const EnsemblePlan* P, int* ti, int* grid, int* nitems) {
    for (int c = 0; c < 2; c++) {
        if (ti) ti[c] = P->ti;
        if (grid) grid[c] = P->grid;
        if (nitems) nitems[c] = P->nclass[c];
    }
}

int ensemble_parity(const EnsemblePlan* P) { return P->parity; }

void ensemble_destroy(EnsemblePlan* P) {
    if (!P) return;
    for (int c = 0; c < 2; c++)
        if (P->exec[c]) hipGraphExecDestroy(P->exec[c]);
    if (P->d_items) hipFree(P->d_items);
    if (P->d_mem) hipFree(P->d_mem);
    if (P->d_cursor) hipFree(P->d_cursor);
    free_budget_rows(*P);
    if (P->cap) hipStreamDestroy(P->cap);
    delete P;
}

}  // namespace monc
