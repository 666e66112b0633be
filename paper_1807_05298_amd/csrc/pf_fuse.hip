// Fusion groups: the stream work of several simulators merged into shared
// launches.
//
// A member simulator records every kernel launch, copy and synchronisation
// of its stream instead of issuing them (pf_internal.h: launch, copy_h2d,
// copy_d2h, stream_sync).  Each member is driven by its own host thread; at
// a synchronisation point the thread waits until every member has reached
// one, and the last to arrive issues the recorded work of all members on the
// group's stream: the k-th launches of the same kernel (with the same block
// size) in the members' queues are issued as one launch (k_multi over a
// table of (member, block range) entries) once every member that has one
// reached it; other operations run one by one.  Every member's operations run in its own order with the same
// arguments, block counts and reductions as alone, so its results do not
// depend on the other members.
#include "pf_internal.h"

#include <algorithm>
#include <condition_variable>
#include <cstring>
#include <map>
#include <mutex>
#include <thread>

namespace pf {

struct Fusion {
    int device = 0;
    hipStream_t stream = nullptr;
    std::mutex mu;
    std::condition_variable cv;
    std::vector<Sim*> members;
    int waiting = 0;                 // members at a synchronisation point
    bool flushing = false;
    uint64_t gen = 0;                // issued batches of recorded work
    std::string err;                 // error of the last issue (every member of it reports it)
    // the merged launches' tables: built in pinned host memory, copied once per issue
    uint8_t* h_tab = nullptr;
    size_t h_cap = 0;
    void* d_tab = nullptr;
    size_t d_cap = 0;
    std::vector<uint8_t> tab;
    int64_t n_issue = 0, n_ops = 0, n_launch = 0;
};

namespace {

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// One planned operation of an issue.
struct Planned {
    MultiFn multi;                   // merged launch, or null: host operation host_op
    unsigned blocks = 0, threads = 0;
    size_t shm = 0, tab_off = 0;
    int count = 0;
    const Op* host_op = nullptr;
};

// An operation's label within an issue: its kernel and block size, and how
// many launches of that kernel precede it in its member's queue.  The k-th
// launches of a kernel in different members' queues are the ones merged.
struct Label {
    MultiFn f;
    uint32_t threads;
    int occ;
    bool operator<(const Label& o) const {
        if (f != o.f) return std::less<MultiFn>()(f, o.f);
        if (threads != o.threads) return threads < o.threads;
        return occ < o.occ;
    }
};

// Issue every member's recorded operations (all members wait).  A label is
// launched once every member whose queue holds it has it at its head (so the
// members that reach it later are not left to a launch of their own); when
// no label is complete (the heads wait on one another), the one that the
// fewest members still have to reach goes first.  Host operations run when they
// reach their member's head.
void issue(Fusion& F, const std::vector<Sim*>& mem) {
    const size_t n = mem.size();
    std::vector<size_t> head(n, 0);
    std::vector<std::vector<int>> lab(n);        // label index of every operation (-1: host)
    std::vector<Label> labels;
    std::vector<int> need, at;                   // members holding each label, members with it at their head
    {
        std::map<Label, int> index;
        std::map<std::pair<MultiFn, uint32_t>, int> occ;
        for (size_t i = 0; i < n; ++i) {
            occ.clear();
            lab[i].resize(mem[i]->ops.size());
            for (size_t k = 0; k < mem[i]->ops.size(); ++k) {
                const Op& o = mem[i]->ops[k];
                if (!o.multi) {
                    lab[i][k] = -1;
                    continue;
                }
                const Label L{o.multi, o.threads, occ[{o.multi, o.threads}]++};
                auto it = index.find(L);
                if (it == index.end()) {
                    it = index.emplace(L, (int)labels.size()).first;
                    labels.push_back(L);
                    need.push_back(0);
                    at.push_back(0);
                }
                lab[i][k] = it->second;
                need[it->second]++;
            }
        }
    }
    std::vector<int> ready;                      // complete labels
    auto arrive = [&](size_t i) {
        if (head[i] >= lab[i].size()) return;
        const int l = lab[i][head[i]];
        if (l >= 0 && ++at[l] == need[l]) ready.push_back(l);
    };
    for (size_t i = 0; i < n; ++i) arrive(i);
    std::vector<Planned> plan;
    std::vector<int> grp;
    F.tab.clear();
    size_t left_total = 0;
    for (size_t i = 0; i < n; ++i) left_total += lab[i].size();
    while (left_total > 0) {
        // host operations at the heads first: they merge with nothing
        bool host = false;
        for (size_t i = 0; i < n; ++i)
            while (head[i] < lab[i].size() && lab[i][head[i]] < 0) {
                Planned p{};
                p.host_op = &mem[i]->ops[head[i]];
                plan.push_back(p);
                F.n_ops++;
                head[i]++;
                left_total--;
                arrive(i);
                host = true;
            }
        if (host) continue;
        int l = -1;
        if (!ready.empty()) {
            l = ready.back();
            ready.pop_back();
        } else {
            // the heads wait on one another: the label fewest members still
            // have to reach (then the one at the most heads, then the member
            // with the most operations left)
            size_t most = 0;
            for (size_t i = 0; i < n; ++i) {
                if (head[i] >= lab[i].size()) continue;
                const int c = lab[i][head[i]];
                const size_t left = lab[i].size() - head[i];
                const int dc = need[c] - at[c], dl = l < 0 ? 0 : need[l] - at[l];
                if (l < 0 || dc < dl || (dc == dl && (at[c] > at[l] || (at[c] == at[l] && left > most)))) {
                    l = c;
                    most = left;
                }
            }
        }
        grp.clear();
        for (size_t j = 0; j < n; ++j)
            if (head[j] < lab[j].size() && lab[j][head[j]] == l) grp.push_back((int)j);
        const Op& o = mem[grp[0]]->ops[head[grp[0]]];
        Planned p{};
        p.multi = o.multi;
        p.threads = o.threads;
        // [first blocks of the entries][entries]: the entries of one launch are
        // contiguous (k_multi indexes them as an array: the same kernel, so the
        // same entry type and size)
        p.tab_off = align_up(F.tab.size(), 256);
        const size_t ent = p.tab_off + multi_entries((int)grp.size());
        F.tab.resize(ent + grp.size() * o.len);
        uint32_t b0 = 0;
        for (size_t g = 0; g < grp.size(); ++g) {
            const int j = grp[g];
            const Op& q = mem[j]->ops[head[j]];
            std::memcpy(F.tab.data() + p.tab_off + 4 * g, &b0, sizeof(b0));
            std::memcpy(F.tab.data() + ent + g * o.len, mem[j]->op_bytes.data() + q.off, q.len);
            b0 += (uint32_t)align_up(q.nb, 8);
            p.shm = std::max(p.shm, q.shm);
            F.n_ops++;
            head[j]++;
            left_total--;
        }
        at[l] -= (int)grp.size();
        need[l] -= (int)grp.size();
        p.count = (int)grp.size();
        p.blocks = b0;
        plan.push_back(p);
        for (int j : grp) arrive((size_t)j);
    }
    // tables to the device in one copy, then the operations in plan order
    const size_t bytes = F.tab.size();
    if (bytes > 0) {
        if (bytes > F.h_cap) {
            if (F.h_tab) PF_HIP(hipHostFree(F.h_tab));
            F.h_tab = nullptr;
            F.h_cap = align_up(bytes * 2, 1 << 16);
            PF_HIP(hipHostMalloc((void**)&F.h_tab, F.h_cap, hipHostMallocDefault));
        }
        if (bytes > F.d_cap) {
            if (F.d_tab) PF_HIP(hipFree(F.d_tab));
            F.d_tab = nullptr;
            F.d_cap = align_up(bytes * 2, 1 << 16);
            PF_HIP(hipMalloc(&F.d_tab, F.d_cap));
        }
        std::memcpy(F.h_tab, F.tab.data(), bytes);
        PF_HIP(hipMemcpyAsync(F.d_tab, F.h_tab, bytes, hipMemcpyHostToDevice, F.stream));
    }
    for (const Planned& p : plan) {
        if (p.multi && p.blocks == 0) continue;
        if (p.multi) {
            p.multi(static_cast<const uint8_t*>(F.d_tab) + p.tab_off, p.count, p.blocks, p.threads, p.shm, F.stream);
            PF_LAUNCH_CHECK();
            F.n_launch++;
        } else {
            p.host_op->host(F.stream);
            PF_LAUNCH_CHECK();
            F.n_launch++;
        }
    }
    PF_HIP(hipStreamSynchronize(F.stream));
    F.n_issue++;
}

// Called with the lock held when every member waits: issue their work with
// the lock released, then release them.
void issue_all(Fusion& F, std::unique_lock<std::mutex>& lk) {
    F.flushing = true;
    const std::vector<Sim*> mem = F.members;
    lk.unlock();
    std::string err;
    try {
        issue(F, mem);
    } catch (const HipError& e) {
        err = e.msg;
    } catch (const std::exception& e) {
        err = e.what();
    }
    for (Sim* m : mem) {
        m->ops.clear();
        m->op_bytes.clear();
    }
    lk.lock();
    F.flushing = false;
    F.waiting = 0;
    F.err = err;
    ++F.gen;
    F.cv.notify_all();
}

// Remove a member that has nothing recorded.
void drop(Sim& s) {
    Fusion& F = *s.fu;
    std::unique_lock<std::mutex> lk(F.mu);
    F.cv.wait(lk, [&] { return !F.flushing; });
    F.members.erase(std::find(F.members.begin(), F.members.end(), &s));
    s.fu = nullptr;
    // the others may all be waiting for this member
    if (!F.members.empty() && F.waiting == (int)F.members.size()) issue_all(F, lk);
}

void leave(Sim& s) {
    std::string err;
    try {
        fusion_sync(s);
    } catch (const HipError& e) {
        err = e.msg;
    }
    drop(s);
    if (!err.empty()) throw HipError{err};
}

}  // namespace

void fusion_record(Sim& s, MultiFn f, uint32_t nb, uint32_t threads, size_t shm, const void* entry, size_t len) {
    Op op;
    op.multi = f;
    op.nb = nb;
    op.threads = threads;
    op.shm = shm;
    op.off = align_up(s.op_bytes.size(), 16);
    op.len = len;
    s.op_bytes.resize(op.off + len);
    std::memcpy(s.op_bytes.data() + op.off, entry, len);
    s.ops.push_back(std::move(op));
}

void fusion_host(Sim& s, std::function<void(hipStream_t)> fn) {
    Op op;
    op.host = std::move(fn);
    s.ops.push_back(std::move(op));
}

void fusion_sync(Sim& s) {
    Fusion& F = *s.fu;
    std::unique_lock<std::mutex> lk(F.mu);
    const uint64_t g = F.gen;
    ++F.waiting;
    if (F.waiting == (int)F.members.size()) issue_all(F, lk);
    else F.cv.wait(lk, [&] { return F.gen != g; });
    if (!F.err.empty()) throw HipError{F.err};
}

void copy_h2d(Sim& s, void* dst, const void* src, size_t bytes) {
    if (!bytes) return;
    if (!s.fu) {
        PF_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s.stream));
        return;
    }
    // the source is copied now: the caller's buffer may change before the issue
    auto data = std::make_shared<std::vector<uint8_t>>((const uint8_t*)src, (const uint8_t*)src + bytes);
    // (the operation, and so the copy's source, lives until the issue has synchronised)
    fusion_host(s, [dst, data](hipStream_t q) {
        PF_HIP(hipMemcpyAsync(dst, data->data(), data->size(), hipMemcpyHostToDevice, q));
    });
}

void copy_d2h(Sim& s, void* dst, const void* src, size_t bytes) {
    if (!bytes) return;
    if (!s.fu) {
        PF_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s.stream));
        return;
    }
    // dst stays valid: the member waits at its next synchronisation point
    fusion_host(s, [dst, src, bytes](hipStream_t q) {
        PF_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, q));
    });
}

void stream_sync(Sim& s) {
    if (s.fu) fusion_sync(s);
    else PF_HIP(hipStreamSynchronize(s.stream));
}

}  // namespace pf

struct pf_fusion {
    pf::Fusion f;
};

namespace {

using pf::HipError;
using pf::set_error;

}  // namespace

extern "C" {

pf_status pf_fusion_create(void* hip_stream, pf_fusion** out) {
    if (!out) {
        set_error("null output handle");
        return PF_EINVAL;
    }
    pf_fusion* h = new pf_fusion();
    if (hipGetDevice(&h->f.device) != hipSuccess) {
        delete h;
        set_error("hipGetDevice failed");
        return PF_EHIP;
    }
    if (hip_stream) {
        int sdev = -1;
        if (hipStreamGetDevice((hipStream_t)hip_stream, &sdev) != hipSuccess || sdev != h->f.device) {
            delete h;
            set_error("the stream belongs to another device than the current one");
            return PF_EINVAL;
        }
    }
    h->f.stream = (hipStream_t)hip_stream;
    *out = h;
    return PF_OK;
}

pf_status pf_fusion_join(pf_fusion* h, pf_sim* sim) {
    if (!h || !sim) {
        set_error("null argument");
        return PF_EINVAL;
    }
    pf::Sim& s = pf_sim_state(sim);
    if (s.fu) {
        set_error("the simulator is already in a fusion group");
        return PF_EINVAL;
    }
    if (s.device != h->f.device) {
        set_error("the simulator and the fusion group are on different devices");
        return PF_EINVAL;
    }
    if (s.static_dev >= 0 || s.prof_id != 0) {
        set_error("a simulator on the static workspace or with kernel timing on cannot join a fusion group");
        return PF_EINVAL;
    }
    // the simulator's own stream (and its side stream) are done with its earlier work
    if (hipStreamSynchronize(s.stream) != hipSuccess || (s.aux && hipStreamSynchronize(s.aux) != hipSuccess)) {
        set_error("hipStreamSynchronize failed");
        return PF_EHIP;
    }
    s.coarse_pending = false;
    pf::Fusion& F = h->f;
    std::unique_lock<std::mutex> lk(F.mu);
    F.cv.wait(lk, [&] { return !F.flushing; });
    F.members.push_back(&s);
    s.fu = &F;
    return PF_OK;
}

pf_status pf_fusion_leave(pf_sim* sim) {
    if (!sim) {
        set_error("null argument");
        return PF_EINVAL;
    }
    pf::Sim& s = pf_sim_state(sim);
    if (!s.fu) return PF_OK;
    try {
        pf::leave(s);
    } catch (const HipError& e) {
        set_error(e.msg);
        return PF_EHIP;
    }
    return PF_OK;
}

pf_status pf_fusion_stats(pf_fusion* h, int64_t* issues, int64_t* ops, int64_t* launches) {
    if (!h) {
        set_error("null argument");
        return PF_EINVAL;
    }
    std::lock_guard<std::mutex> lk(h->f.mu);
    if (issues) *issues = h->f.n_issue;
    if (ops) *ops = h->f.n_ops;
    if (launches) *launches = h->f.n_launch;
    return PF_OK;
}

pf_status pf_fusion_step(pf_fusion* h, int32_t n, pf_sim* const* sims, const double* dts, pf_step_stats* stats) {
    if (!h || n < 1 || !sims || !dts) {
        set_error("bad fusion step arguments");
        return PF_EINVAL;
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < i; ++j)
            if (!sims[i] || sims[i] == sims[j]) {
                set_error("null or repeated simulator");
                return PF_EINVAL;
            }
    // every simulator joins before any steps, so that the first issue already
    // covers all of them (a thread of its own would join after the first
    // threads' first synchronisation points)
    for (int i = 0; i < n; ++i) {
        const pf_status sj = pf_fusion_join(h, sims[i]);
        if (sj != PF_OK) {
            const std::string m = pf_last_error();
            for (int k = 0; k < i; ++k) pf::drop(pf_sim_state(sims[k]));    // nothing recorded yet
            set_error("simulator " + std::to_string(i) + ": " + m);
            return sj;
        }
    }
    std::vector<pf_status> st(n, PF_OK);
    std::vector<std::string> msg(n);
    std::vector<std::thread> th;
    th.reserve(n);
    for (int i = 0; i < n; ++i)
        th.emplace_back([&, i] {
            (void)hipSetDevice(h->f.device);
            st[i] = pf_step(sims[i], dts[i], stats ? stats + i : nullptr);
            if (st[i] != PF_OK) msg[i] = pf_last_error();
            const pf_status sl = pf_fusion_leave(sims[i]);
            if (st[i] == PF_OK && sl != PF_OK) {
                st[i] = sl;
                msg[i] = pf_last_error();
            }
        });
    for (auto& t : th) t.join();
    for (int i = 0; i < n; ++i)
        if (st[i] != PF_OK) {
            set_error("simulator " + std::to_string(i) + ": " + msg[i]);
            return st[i];
        }
    return PF_OK;
}

void pf_fusion_destroy(pf_fusion* h) {
    if (!h) return;
    {
        std::lock_guard<std::mutex> lk(h->f.mu);
        if (!h->f.members.empty()) {
            set_error("pf_fusion_destroy: the group still has members (not destroyed)");
            return;
        }
    }
    if (h->f.h_tab) (void)hipHostFree(h->f.h_tab);
    if (h->f.d_tab) (void)hipFree(h->f.d_tab);
    delete h;
}

}  // extern "C"
