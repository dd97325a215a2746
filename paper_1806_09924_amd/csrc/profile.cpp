#include "profile.h"

#include <map>
#include <mutex>
#include <string>
#include <vector>

namespace fr {
namespace {

struct Pair {
    hipEvent_t a = nullptr, b = nullptr;
    bool closed = false;                          // b recorded (the scope has ended)
};

struct Entry {
    std::string name;
    std::vector<Pair> ev;
    double bytes = 0.0;
    double ms = 0.0;
    int64_t launches = 0;
};

std::mutex g_mu;
bool g_on = false;
std::vector<Entry> g_entries;
std::map<std::string, int> g_index;
std::vector<hipEvent_t> g_pool;

hipEvent_t take_event() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

// Folds the closed event pairs of an entry into its totals and returns their events to the
// pool; pairs of scopes still open (another thread) stay.  Errors of these calls are
// cleared so that they do not surface at a later launch check.
void drain(Entry& e) {
    std::vector<Pair> open;
    for (auto& p : e.ev) {
        if (!p.closed) {
            open.push_back(p);
            continue;
        }
        float ms = 0.0f;
        if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess)
            e.ms += double(ms);
        else
            (void)hipGetLastError();
        g_pool.push_back(p.a);
        g_pool.push_back(p.b);
    }
    e.ev.swap(open);
}

}  // namespace

bool prof_enabled() { return g_on; }

void prof_enable(bool on) {
    std::lock_guard<std::mutex> lk(g_mu);
    for (auto& e : g_entries) drain(e);
    g_entries.clear();
    g_index.clear();
    g_on = on;
}

// Each scope owns its event pair, so scopes of one name may overlap (two host threads).
ProfScope::ProfScope(const char* name, hipStream_t stream, double bytes) {
    if (!g_on) return;
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_index.find(name);
    if (it == g_index.end()) {
        g_index[name] = int(g_entries.size());
        g_entries.push_back(Entry{name, {}, 0.0, 0.0, 0});
        it = g_index.find(name);
    }
    idx = it->second;
    s = stream;
    Entry& e = g_entries[size_t(idx)];
    if (e.ev.size() >= 16384) drain(e);   // bounded event pool; folding synchronises
    a = take_event();
    b = take_event();
    (void)hipEventRecord(a, s);
    e.ev.push_back(Pair{a, b, false});
    e.bytes += bytes;
    e.launches += 1;
}

ProfScope::~ProfScope() {
    if (idx < 0) return;
    std::lock_guard<std::mutex> lk(g_mu);
    (void)hipEventRecord(b, s);
    if (size_t(idx) >= g_entries.size()) return;   // registry reset while the scope was open
    auto& ev = g_entries[size_t(idx)].ev;
    for (auto p = ev.rbegin(); p != ev.rend(); ++p)
        if (p->a == a) {
            p->closed = true;
            break;
        }
}

int prof_count() {
    std::lock_guard<std::mutex> lk(g_mu);
    return int(g_entries.size());
}

bool prof_read(int i, const char** name, int64_t* launches, double* ms, double* bytes) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (i < 0 || size_t(i) >= g_entries.size()) return false;
    Entry& e = g_entries[size_t(i)];
    drain(e);
    if (name) *name = e.name.c_str();
    if (launches) *launches = e.launches;
    if (ms) *ms = e.ms;
    if (bytes) *bytes = e.bytes;
    return true;
}

}  // namespace fr
