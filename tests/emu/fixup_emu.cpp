// CPU-thread emulator of the Stream-K fix-up protocol (test infrastructure).
//
// One std::thread per workgroup walks its segments of a schedule (records in
// the format of skgemm_schedule) and exchanges partial tiles with its peers
// through a shared slot array and ready flags, as the GPU kernel does:
//  * owner fix-up (basic Stream-K algorithm, Wait/Signal): a segment that does
//    not start its tile stores its partial into slot wg and raises flag wg; the
//    tile's owner waits for the flags of its peers in ascending order, adds
//    their partials, writes C and clears the flags for the next launch;
//  * split fix-up: every tile is cut into s one-segment shares held by s
//    consecutive workgroups; units u of a tile go to reducer u mod R
//    (R = min(s, units)); each contributor stores the units it does not
//    reduce and raises one flag word per other reducer; each reducer waits
//    for its word from every other contributor, adds their copies, writes its
//    units and clears the words it waited on.
// Flags are std::atomic with release stores and acquire loads (the ordering
// the device code builds from coherent stores, a wait for their completion,
// and the flag store); slots are plain memory, so ThreadSanitizer reports
// any read of a slot that the protocol does not order after its write.
//
// Each MAC-loop iteration (tile, k) contributes the integer value
// tile * 4096 + k + 1 to every unit of its tile, so any dropped, doubled or
// misplaced partial changes C.  Several launches reuse the slots and flags
// (threads joined in between, as kernel boundaries).
//
// stdin:  grid coop_s units launches spin_limit drop_wg skip_wait
//         then one record per line: wg seq tile lo hi role first_peer last_peer
// exit:   0 all tiles exact, 1 wrong result, 2 bad input, 3 a wait timed out
#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <vector>

namespace {

struct Rec { int wg, seq, tile, lo, hi, role, p0, p1; };
enum { FULL = 0, PARTIAL = 1, OWNER = 2 };
constexpr int kWords = 8;

int g_grid, g_coop, g_units, g_launches, g_drop, g_skip;
long g_spin;
std::vector<std::vector<Rec>> g_segs;        // per workgroup, in order
std::vector<double> g_slots;                 // grid x units
std::vector<std::atomic<int>> g_flags;       // grid x kWords
std::vector<double> g_C;                     // tiles x units
std::atomic<int> g_err{0};

double contrib(int tile, int lo, int hi) {
    double s = 0;
    for (int k = lo; k < hi; ++k) s += double(tile) * 4096.0 + k + 1;
    return s;
}

// Bounded wait for word w of flag line k; false (and the error word set) on timeout.
bool wait_flag(int k, int w) {
    for (long i = 0; i < g_spin; ++i) {
        if (g_flags[size_t(k) * kWords + w].load(std::memory_order_acquire) != 0) return true;
        std::this_thread::yield();
    }
    g_err.store(1, std::memory_order_relaxed);
    return false;
}

void raise_flag(int wg, int w) {
    if (wg == g_drop) return;                 // a dropped signal (tests the timeout)
    g_flags[size_t(wg) * kWords + w].store(1, std::memory_order_release);
}

void workgroup(int wg) {
    for (const Rec& r : g_segs[wg]) {
        const double acc = contrib(r.tile, r.lo, r.hi);
        std::vector<double> units(g_units, acc);
        const bool split = g_coop >= 2 && r.role != FULL;
        if (split) {
            const int s = g_coop, c = wg % s, first = wg - c, R = s < g_units ? s : g_units;
            // store the units this contributor does not reduce, one word per other reducer
            for (int u = 0; u < g_units; ++u)
                if (u % R != c) g_slots[size_t(wg) * g_units + u] = units[u];
            for (int q = 0; q < R; ++q)
                if (q != c) raise_flag(wg, q);
            if (c >= R) continue;
            std::vector<int> waited;
            for (int k = first; k < first + s; ++k) {
                if (k == wg) continue;
                if (!g_skip && !wait_flag(k, c)) break;
                waited.push_back(k);
                for (int u = c; u < g_units; u += R) units[u] += g_slots[size_t(k) * g_units + u];
            }
            for (int u = c; u < g_units; u += R) g_C[size_t(r.tile) * g_units + u] = units[u];
            for (int k : waited) g_flags[size_t(k) * kWords + c].store(0, std::memory_order_relaxed);
            continue;
        }
        if (r.role == FULL) {
            for (int u = 0; u < g_units; ++u) g_C[size_t(r.tile) * g_units + u] = units[u];
        } else if (r.role == PARTIAL) {
            for (int u = 0; u < g_units; ++u) g_slots[size_t(wg) * g_units + u] = units[u];
            raise_flag(wg, 0);
        } else {
            std::vector<int> waited;
            for (int k = r.p0; k <= r.p1; ++k) {
                if (!g_skip && !wait_flag(k, 0)) break;
                waited.push_back(k);
                for (int u = 0; u < g_units; ++u) units[u] += g_slots[size_t(k) * g_units + u];
            }
            for (int u = 0; u < g_units; ++u) g_C[size_t(r.tile) * g_units + u] = units[u];
            for (int k : waited) g_flags[size_t(k) * kWords].store(0, std::memory_order_relaxed);
        }
    }
}

}  // namespace

int main() {
    if (std::scanf("%d %d %d %d %ld %d %d", &g_grid, &g_coop, &g_units, &g_launches, &g_spin, &g_drop, &g_skip) != 7 ||
        g_grid <= 0 || g_units <= 0 || g_units > kWords || g_launches <= 0)
        return 2;
    g_segs.assign(g_grid, {});
    int tiles = 0;
    Rec r;
    while (std::scanf("%d %d %d %d %d %d %d %d", &r.wg, &r.seq, &r.tile, &r.lo, &r.hi, &r.role, &r.p0, &r.p1) == 8) {
        if (r.wg < 0 || r.wg >= g_grid || r.seq != int(g_segs[r.wg].size())) return 2;
        g_segs[r.wg].push_back(r);
        if (r.tile + 1 > tiles) tiles = r.tile + 1;
    }
    // expected C per tile: the sum over all its iterations
    std::vector<int> ipt(tiles, 0);
    for (auto& v : g_segs)
        for (auto& s : v)
            if (s.hi > ipt[s.tile]) ipt[s.tile] = s.hi;
    g_slots.assign(size_t(g_grid) * g_units, 0.0);
    g_flags = std::vector<std::atomic<int>>(size_t(g_grid) * kWords);
    for (auto& f : g_flags) f.store(0);
    int status = 0;
    for (int l = 0; l < g_launches && status == 0; ++l) {
        g_C.assign(size_t(tiles) * g_units, -1.0);
        std::vector<std::thread> th;
        for (int x = 0; x < g_grid; ++x) th.emplace_back(workgroup, x);
        for (auto& t : th) t.join();
        if (g_err.load()) {
            std::printf("launch %d: a fix-up wait timed out\n", l);
            return 3;
        }
        for (int t = 0; t < tiles; ++t)
            for (int u = 0; u < g_units; ++u)
                if (g_C[size_t(t) * g_units + u] != contrib(t, 0, ipt[t])) {
                    std::printf("launch %d: tile %d unit %d wrong\n", l, t, u);
                    status = 1;
                }
        for (auto& f : g_flags)
            if (f.load() != 0) {
                std::printf("launch %d: a flag was left raised\n", l);
                status = 1;
                break;
            }
    }
    if (status == 0) std::printf("ok %d launches\n", g_launches);
    return status;
}
