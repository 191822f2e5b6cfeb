// Claim schedule of a persistent launch (see PSeg and PDep in qw_desc.h):
// host code only, shared by the executor and the host-only schedule query.
#include <algorithm>
#include <string>

#include "qw_internal.h"

namespace qw {

std::string persist_schedule(const std::vector<int> &parent, const std::vector<uint32_t> &passes,
                             const std::vector<PersistDesc> &descs, int tile_order, uint32_t chunk_max,
                             uint32_t grid, PersistSchedule *out) {
    const size_t T = parent.size();
    if (passes.size() != T) return "parent and pass counts differ in length";
    if (chunk_max == 0 || (chunk_max & (chunk_max - 1))) return "claim size must be a power of two";
    // level of a descriptor: the passes that must have run before it (its
    // task's earlier passes and, through parents, all of theirs), so that
    // every dependency lies in an earlier level
    std::vector<uint32_t> start(T, 0);
    for (size_t t = 0; t < T; ++t) {
        if (parent[t] < 0) continue;
        const size_t pt = (size_t)parent[t];
        if (pt >= t || passes[pt] == 0) return "a parent task must come first and have passes";
        start[t] = start[pt] + passes[pt];
    }
    size_t total = 0;
    for (uint32_t p : passes) total += p;
    if (descs.size() != total) return "one descriptor per (task, pass) expected";
    std::vector<std::vector<uint32_t>> slot(T);
    for (size_t t = 0; t < T; ++t) slot[t].assign(passes[t], kNoDep);
    for (uint32_t i = 0; i < (uint32_t)descs.size(); ++i) {
        const PersistDesc &d = descs[i];
        if (d.t >= T || d.k >= passes[d.t] || slot[d.t][d.k] != kNoDep) return "descriptors do not cover the tasks' passes once";
        if (d.units == 0 || (d.units & (d.units - 1))) return "units must be a power of two";
        slot[d.t][d.k] = i;
    }
    // claim order: by level, then pass structure, then task
    std::vector<uint32_t> &ord = out->order;
    ord.resize(descs.size());
    for (uint32_t i = 0; i < (uint32_t)ord.size(); ++i) ord[i] = i;
    auto level = [&](uint32_t i) { return start[descs[i].t] + descs[i].k; };
    std::sort(ord.begin(), ord.end(), [&](uint32_t a, uint32_t b) {
        if (level(a) != level(b)) return level(a) < level(b);
        if (descs[a].kind != descs[b].kind) return descs[a].kind < descs[b].kind;
        return descs[a].t < descs[b].t;
    });
    std::vector<uint32_t> pos(descs.size());
    for (uint32_t i = 0; i < (uint32_t)ord.size(); ++i) pos[ord[i]] = i;
    out->segs.clear();
    out->claims = 0;
    for (uint32_t i = 0; i < (uint32_t)ord.size();) {
        uint32_t j = i + 1;
        const PersistDesc &a = descs[ord[i]];
        while (j < ord.size() && level(ord[j]) == level(ord[i]) && descs[ord[j]].kind == a.kind) ++j;
        const uint32_t count = j - i, units = a.units;
        bool shared_src = true, same_units = true;
        for (uint32_t q = i + 1; q < j; ++q) {
            shared_src = shared_src && descs[ord[q]].src == a.src;
            same_units = same_units && descs[ord[q]].units == units;
        }
        if (!same_units) return "descriptors of one pass structure differ in units";
        const bool tmaj = !shared_src && (tile_order == 2 || (tile_order == 1 && a.relabel));
        // up to chunk_max units per claim, keeping at least 4 claims per workgroup
        uint32_t chunk = chunk_max;
        while (chunk > 1 && (units % chunk != 0 || (uint64_t)units * count / chunk < 4ull * grid)) chunk >>= 1;
        PSeg e{};
        e.claim0 = out->claims;
        e.n_claims = units / chunk * count;
        e.desc0 = i;
        e.n_descs = count;
        e.chunk = chunk;
        e.kind = a.kind;
        e.tmaj = tmaj ? 1u : 0u;
        e.units = units;
        out->segs.push_back(e);
        out->claims += e.n_claims;
        i = j;
    }
    // each descriptor waits for its task's previous pass, or for the last
    // pass of its parent task
    out->deps.assign(descs.size(), PDep{kNoDep, 0u});
    for (uint32_t i = 0; i < (uint32_t)descs.size(); ++i) {
        const PersistDesc &d = descs[i];
        uint32_t dep = kNoDep;
        if (d.k > 0)
            dep = slot[d.t][d.k - 1];
        else if (parent[d.t] >= 0)
            dep = slot[(size_t)parent[d.t]].back();
        if (dep != kNoDep) out->deps[pos[i]] = PDep{pos[dep], descs[dep].units};
    }
    return "";
}

}  // namespace qw
