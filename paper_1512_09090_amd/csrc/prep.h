// prep.h - host-side preprocessing of the isochrone library.
//
// Builds, from a plain arc list, everything the query needs (Section 5,
// generic isoPHAST preprocessing plus the CorePHAST step):
//   * a single-level vertex partition (recursive coordinate bisection, or
//     BFS-grown cells, or a caller-given one);
//   * a contraction hierarchy (Section 2) in which the internal vertices of
//     every cell are contracted first, cell by cell, and the uncontracted
//     boundary vertices (the core) are then contracted by a CH of their own;
//   * a sweep layout: core vertices first ordered by descending level, then
//     every cell's internal vertices ordered by descending level;
//   * the downward graph as a CSR over sweep positions, each entry carrying
//     the flags "original arc tail->head" and "original arc head->tail" and,
//     where needed, a dummy entry of length infinity (Section 5, output of
//     isochrone edges during the sweep);
//   * the upward graph for the host upward search;
//   * per core vertex the cell-restricted eccentricity (Section 4 definition,
//     computed as in Section 5) and per cell an "uncovered" mark.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace iso {

constexpr uint32_t INF = 0xFFFFFFFFu;
constexpr uint32_t NO_CELL = 0xFFFFFFFFu;
// downward-graph entry: word0 = tail position | flags, word1 = length
constexpr uint32_t TAIL_MASK = 0x3FFFFFFFu;
constexpr uint32_t FLAG_FWD = 0x80000000u;   // original arc (tail, head) exists
constexpr uint32_t FLAG_REV = 0x40000000u;   // original arc (head, tail) exists

inline uint32_t sat_add(uint32_t a, uint32_t b) {
    uint64_t s = uint64_t(a) + b;
    return s >= INF ? INF : uint32_t(s);
}

struct PrepOptions {
    uint32_t num_cells = 0;          // 0 = no partition
    uint32_t max_cell_size = 2048;
    int threads = 0;
    int verbose = 0;
    // Cell phase: an internal vertex is contracted only while (1000 * shortcuts it needs /
    // arcs it removes) <= cell_max_quot; the others stay in the core (0 = contract all).
    uint64_t cell_max_quot = 2000;
};

struct Prep {
    uint32_t n = 0, n_core = 0, num_cells = 0;
    uint64_t m = 0;               // arcs after simplification
    uint64_t shortcuts = 0;

    std::vector<uint32_t> perm;   // position -> original id
    std::vector<uint32_t> pos;    // original id -> position
    std::vector<uint32_t> cell_of;// original id -> cell (NO_CELL when no partition)

    // downward graph, CSR by head position; entries are (tail_pos | flags, length)
    std::vector<uint32_t> down_off;   // n + 1
    std::vector<uint32_t> down_arc;   // 2 * entries
    // upward graph, CSR by tail position (host only)
    std::vector<uint32_t> up_off;     // n + 1
    std::vector<uint32_t> up_head;
    std::vector<uint32_t> up_w;

    // core levels, top first: level i spans positions [core_lvl[i], core_lvl[i+1])
    std::vector<uint32_t> core_lvl;
    // cell c's internal vertices span [cell_off[c], cell_off[c+1]); its levels (top first)
    // start at cell_lvl[cell_lvl_ptr[c] .. cell_lvl_ptr[c+1])
    std::vector<uint32_t> cell_off;
    std::vector<uint32_t> cell_lvl_ptr;
    std::vector<uint32_t> cell_lvl;
    std::vector<uint32_t> core_cell;  // n_core: cell of each core position (NO_CELL without partition)
    std::vector<uint32_t> core_ecc;   // n_core: eccentricity within the cell (INF if not finite-bounded)
    std::vector<uint8_t> uncovered;   // num_cells

    uint32_t max_cell_internal = 0, max_cell_levels = 0;
    double seconds = 0.0;
};

// Simplified arc list: no self-loops, parallel arcs merged to the minimum weight,
// sorted by (tail, head).
struct ArcList {
    uint32_t n = 0;
    std::vector<uint32_t> tail, head, w;
};
void simplify_arcs(uint32_t n, uint64_t m, const uint32_t *tail, const uint32_t *head,
                   const uint32_t *w, ArcList &out);

// Partitioners (return cell id per vertex; all ids < num_cells).
void partition_bisect(uint32_t n, const double *xy, uint32_t num_cells, std::vector<uint32_t> &cell_of);
void partition_bfs(const ArcList &g, uint32_t max_cell_size, std::vector<uint32_t> &cell_of,
                   uint32_t &num_cells);

// Full preprocessing.  cell_of may be empty (no partition).
void build_prep(const ArcList &g, const std::vector<uint32_t> &cell_of, uint32_t num_cells,
                const PrepOptions &opt, Prep &out);

// Binary save / load with a version, the hash of the input and an FNV-1a checksum.
enum LoadStatus { LOAD_OK = 0, LOAD_MISSING = 1, LOAD_OTHER_INPUT = 2, LOAD_CORRUPT = 3 };
bool save_prep(const std::string &path, const Prep &p, uint64_t input_hash);
LoadStatus load_prep(const std::string &path, Prep &p, uint64_t input_hash);
uint64_t hash_input(const ArcList &g, const std::vector<uint32_t> &cell_of, uint32_t num_cells);

int resolve_threads(int t);

}  // namespace iso
