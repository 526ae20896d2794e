// Host-side setup of the fine-grained Hines solver: compartment numbering,
// level schedule, branch-to-lane assignment and the device tables of the
// solve kernels (paper §4 "distribution ... computed once during the setup
// phase", §5 memory layout, §6 work balancing).  Pure C++17; no HIP.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace hines {

enum Status : int32_t {
  OK = 0,
  ERR_NULL = 1,
  ERR_BAD_OFFSETS = 2,
  ERR_BAD_PARENT = 3,
  ERR_BAD_BRANCHES = 4,
  ERR_NCELLS = 6,
  ERR_OPTION = 7,
  ERR_OOM = 8,
  ERR_HIP = 9,
  ERR_TOO_BIG = 10,
  ERR_NOT_SDD = 11,
  ERR_STATE = 12,
};

struct Options {
  int32_t rebalance_root = 0;      // §6: re-root each cell at its tree centre
  int32_t split_branches = 0;      // §6: per-level split of longer-than-average branches (1: level
                                   // averages over all cells; 2: over the groups of an
                                   // intermediate packing, the outlook of §8)
  int32_t level_balance = 0;       // §8 outlook: packing may move subtrees one level down
  int32_t group_width = 64;        // §4: lanes per group (multiple of 64, <= 1024)
  int32_t cell_order = 0;          // §4 packing order: 0 input, 1 size descending
  int32_t max_group_unknowns = 0;  // packing cap on compartments per group (0: none)
  int32_t host_only = 0;           // build tables only, no device upload
  int32_t keep_tables = 1;         // keep the exported tables after setup
  int32_t bitwise = 0;             // IEEE divisions, unfused updates: equal to the plain algorithm bit for bit
  int32_t scheduler = 1;           // 1: static heavy-path lane schedule when every branch ascends;
                                   // 0: level-synchronous sweeps (paper §3)
  int32_t cell_lanes = 0;          // 1: one lane per cell (streaming kernel) for hines_solve / timestep
  int32_t cell_seq = 0;            // 1: index-order cell lanes for hines_solve
  int32_t resident = 0;            // 1: LDS-resident path-walk kernel for hines_solve
  int32_t cell_cut_percent = 80;   // cell lanes: cut cells longer than this percentage of the mean
  int32_t cell_max_cuts = 3;       // cell lanes: cut-off subtrees per cell
  int32_t res_pack = 1400;         // resident: compartments per group of consecutive cells
};

// Static chunk schedule (flow kernel): one lane eliminates kFlowChunk
// compartments of one path per chunk step; kSchedLanes lanes per group; at
// most kMaxSteps chunk steps per sweep.
constexpr int32_t kSchedLanes = 64;
constexpr int32_t kMaxSteps = 16384;
constexpr int32_t kFlowChunk = 8;
// LDS block of one lane-chunk: kFlowChunk entries of d, u, b (3 doubles each)
// and one spare double, so that consecutive blocks start in different banks.
constexpr int32_t kFlowBlock8 = 3 * kFlowChunk + 1;
// after the blocks: one identity block read by idle lanes (d = 1, u = 0,
// b = 0 per entry) and a write-only sink: idle lane l writes entry j of a step
// at 8-byte unit l + 3 j of the sink, so no two lanes of one write collide
constexpr int32_t kFlowSink8 = 64 + 3 * kFlowChunk;
constexpr int32_t kFlowTail8 = kFlowBlock8 + kFlowSink8;

// LDS image of a group: d, u, b per slot (nimg slots; 0 when the compartment
// arrays live in the global workspace), two elimination contributions per
// branch, the branch records and a table of level or lane offsets.  Every
// region starts 16-byte aligned.
struct LdsLayout {
  int32_t nimg, nbr_pad, nlev;
  constexpr int64_t u_off() const { return nimg; }  // doubles
  constexpr int64_t b_off() const { return 2 * (int64_t)nimg; }
  constexpr int64_t cd_off() const { return 3 * (int64_t)nimg; }
  constexpr int64_t cb_off() const { return 3 * (int64_t)nimg + nbr_pad; }
  constexpr int64_t br_off_bytes() const { return 8 * (3 * (int64_t)nimg + 2 * (int64_t)nbr_pad); }
  constexpr int64_t tab_off_bytes() const { return br_off_bytes() + 16 * (int64_t)nbr_pad; }
  constexpr int64_t bytes() const {
    const int64_t ints = (int64_t)nlev + 1 > kSchedLanes + 1 ? (int64_t)nlev + 1 : kSchedLanes + 1;
    return (tab_off_bytes() + 4 * ints + 15) & ~(int64_t)15;
  }
};
constexpr int64_t kLdsLimitBytes = 160 * 1024;  // gfx950 LDS per workgroup

// Table ids for export (shared with the C-ABI).
enum TableId : int32_t {
  T_NODE_PLAN = 0,        // int64[n]
  T_BRANCHES = 1,         // int64[nb*8]: cell, level, first, dir, len, parent, group, rank
  T_U_SRC = 2,            // int64[n] in plan order
  T_GROUP_OFFSETS = 3,    // int64[ngroups+1]
  T_GROUP_CELLS = 4,      // int64[ncells]
  T_GROUP_SEG_OFFSETS = 5,  // int64[ngroups+1]
  T_SEG_OFFSETS = 6,      // int64[nseg+1]
  T_LANES = 7,            // int64[nb]
  T_FLOW_GROUPS = 8,      // int64[ngroups*6]: step_off, pos_off, aux_off, nstep, nelem, naux
  T_FLOW_MASKS = 9,       // int64[2*steps]: active and push masks (bit patterns)
  T_FLOW_POS = 10,        // int64[elements]: position | 0x8000 for cell roots
  T_FLOW_AUX = 11,        // int64[pushes]: parent position
  T_CELL_WAVES = 12,      // int64[nwaves*3]: chunk_off, nchunk, ncell
  T_CELL_LANES = 13,      // int64[nwaves*64]: cell of each lane (-1: empty)
  T_CELL_POS = 14,        // int64[nchunks*kCellChunkElems]: [chunk][staging lane][slot] relative position
  T_CELL_FLAGS = 15,      // int64[nchunks*kCellChunkElems]: [chunk][cell lane][element] flags
  T_CELL_MBSRC = 16,      // int64[nwaves*64]: mailbox source lanes (6 bits each), backward | forward << 32
  T_RES_GROUPS = 17,      // int64[ngroups*16]: lo, blob, nslot, ndma, first, count, nchunk, blob_units, nroot,
                          // npath, nlist, rec_off, list_off, cls, steps per chunk, nflip
  T_CELL_RANGE = 18,      // int64[nwaves*64]: first step of the lane's walk | end step << 32 (padding outside)
  T_RES_BLOB = 19,        // int64[blob bytes / 2]: the blobs as uint16 words
  T_SEQ_WAVES = 20,       // int64[nwaves*3]: chunk_off, nchunk, ncell (index-order lanes)
  T_SEQ_LANES = 21,       // int64[nwaves*64]: cell of each lane (-1: empty)
  T_SEQ_POS = 22,         // int64[nchunks*kSeqChunkElems]: [chunk][staging lane][slot] relative position
  T_SEQ_CODE = 23,        // int64[nchunks*kSeqChunkElems]: [chunk][cell lane][element] step code
  T_SEQ_MBSRC = 24,       // int64[nwaves*64]: mailbox source lanes, backward | forward << 32
  T_NUM = 25,
};

// Cell-lane kernel (one lane per cell, or per half of a long cell).  Each cell is processed in a depth-
// first order of its compartments in which the children of a compartment are
// visited with the child needing the deepest contribution stack last (paper
// §2's elimination needs only that children precede parents in the backward
// sweep).  Backward sweep: reverse of that order; forward sweep: the order.
// A wave holds 64 cells of similar size; lane c walks cell c.  Per chunk of
// kCellChunk consecutive steps the table gives, for the staging mapping (lane
// j, slot r) -> (cell lane kCellSlotCells r + j / kCellChunk, element
// j % kCellChunk), the position of the element relative to its cell's first
// compartment, and per (cell lane, element) the flags below.
constexpr int32_t kCellChunk = 16;                     // steps per chunk (a power of two, <= 16)
constexpr int32_t kCellSlotCells = 64 / kCellChunk;     // cells per gather slot
constexpr int32_t kCellChunkElems = 64 * kCellChunk;    // table entries per chunk
// Table index of element e of the cell in lane c: in the gather order (lane j,
// slot r) and in the cell-lane order.
constexpr int64_t cell_pos_index(int64_t chunk, int32_t c, int32_t e) {
  return chunk * kCellChunkElems + (int64_t)((c % kCellSlotCells) * kCellChunk + e) * kCellChunk + c / kCellSlotCells;
}
constexpr int64_t cell_flag_index(int64_t chunk, int32_t c, int32_t e) {
  return chunk * kCellChunkElems + (int64_t)c * kCellChunk + e;
}
constexpr int32_t kCellStack = 12;           // LDS stack slots per lane; slot 0 is a dummy
constexpr int32_t kCellMaxCuts = 3;          // cut-off subtrees per cell (lanes per cell: up to 4)
constexpr uint16_t kCellPadPos = 0xFFFF;     // padding element: no user compartment
constexpr int64_t kCellMaxSize = 65535;      // positions fit 16 bits below kCellPadPos
enum : uint8_t {
  CF_TIP = 1,     // no children: the elimination carry does not enter
  CF_POP = 2,     // two or more children: the stacked contributions of all but the first enter
  CF_PUSH = 4,    // last child of its parent (two or more children): its contribution opens a stack entry
  CF_MERGE = 8,   // middle child: its contribution is added to the top entry
  CF_PAD = 16,    // padding: identity row
  CF_ROOT = 32,   // cell root: no coupling to a parent
  CF_MBOUT = 64,  // root of a cut-off subtree (lane c): its contribution leaves through mailbox c,
                  // x of its parent comes back through it
  CF_MBIN = 128,  // parent of such a root: takes the contribution from the next mailbox of its
                  // lane's source list and returns its x there
};
struct KCellWave {
  int64_t chunk_off;  // first chunk of the wave in the pos / flags / scratch tables
  int32_t nchunk;     // chunks per sweep
  int32_t ncell;      // occupied lanes
};
static_assert(sizeof(KCellWave) == 16, "layout");

struct CellLanes {
  bool built = false;
  int64_t nwaves = 0, nchunks = 0;
  int32_t max_need = 0;             // deepest stack of any cell (entries)
  std::vector<KCellWave> waves;     // [nwaves], largest cells first
  std::vector<int32_t> lane_cell;   // [nwaves*64] cell of each lane, -1 for empty lanes
  std::vector<int64_t> base;        // [nwaves*64] first user index of the lane's cell (0: empty)
  std::vector<uint16_t> pos;        // [nchunks*kCellChunkElems] staging order
  std::vector<uint8_t> flags;       // [nchunks*kCellChunkElems] cell-lane order
  std::vector<uint64_t> mbsrc;      // [nwaves*64] mailbox source lanes in the order the lane's
                                    // backward sweep takes them (6 bits each), and in the order
                                    // of its forward sweep << 32; 0 for lanes without takes
  std::vector<uint64_t> range;      // [nwaves*64] steps [q0, q1) of the lane's walk: q0 | q1 << 32;
                                    // every other step of the lane is padding (0 for empty lanes)
};

// Build the cell-lane tables.  parent / cell_offsets must already be valid.
// ERR_TOO_BIG if a cell has more than kCellMaxSize compartments or needs more
// than kCellStack stack entries.
// cut_percent: cells longer than this percentage of the mean cell are cut
// (80 by default); max_cuts: cut-off subtrees per cell, 1 .. kCellMaxCuts.
Status build_cell_lanes(const int32_t* parent, int64_t n, const int64_t* cell_offsets, int64_t ncells,
                        CellLanes& out, std::string& err, int32_t cut_percent = 80,
                        int32_t max_cuts = kCellMaxCuts);

// Index-order cell lanes (option cell_lanes 2).  Same one-lane-per-cell
// elimination, but a lane walks its piece of a cell in decreasing user index in
// the backward sweep.  The parent of every compartment has a lower index (the
// numbering §2 requires), so that order puts children before parents, and a
// cell numbered level by level is read in a few long runs of consecutive
// compartments, whole memory lines, instead of one short branch at a time.  A
// contribution whose parent is not the next step waits in a per-lane LDS slot
// from the first child that adds into it to the parent's step (slots assigned
// by interval colouring); the forward sweep sends the parent's x back to the
// same children through the same slot.  A lane whose index walk would need
// more than kSeqSlots slots walks depth-first instead (the slot code serves
// any children-first order).  Runs of kSeqMinRun or more compartments start
// so that every chunk pair covers one 128-byte line of the user arrays (when
// the arrays start on 128-byte boundaries); a cell much longer than the mean is
// cut into up to kCellMaxCuts + 1 pieces (the longest piece cut again while it
// stays long) on adjacent lanes of one wave, the contribution of each cut-off
// subtree's root crossing through its lane's mailbox as in the cell-lane
// kernel.
constexpr int32_t kSeqChunk = 8;                       // steps per chunk
constexpr int32_t kSeqSlotCells = 64 / kSeqChunk;      // cells per gather slot
constexpr int32_t kSeqChunkElems = 64 * kSeqChunk;     // table entries per chunk
constexpr int32_t kSeqSlots = 26;                      // LDS contribution slots per lane
constexpr int32_t kSeqLine = 16;                       // compartments per 128-byte line
constexpr int32_t kSeqMinRun = 16;                     // runs this long start line-aligned
constexpr int64_t seq_pos_index(int64_t chunk, int32_t c, int32_t e) {
  return chunk * kSeqChunkElems + (int64_t)((c % kSeqSlotCells) * kSeqChunk + e) * kSeqChunk + c / kSeqSlotCells;
}
constexpr int64_t seq_code_index(int64_t chunk, int32_t c, int32_t e) {
  return chunk * kSeqChunkElems + (int64_t)c * kSeqChunk + e;
}
enum : uint16_t {
  SQ_SLOT = 31,         // bits 0-4: slot the step's contribution goes into (0: none)
  SQ_READ_SHIFT = 5,    // bits 5-9: slot holding the contributions of the step's other children
  SQ_TIP = 1 << 10,     // the previous step's contribution does not enter
  SQ_PAD = 1 << 11,     // padding: identity row
  SQ_MBOUT = 1 << 12,   // root of the cut-off subtree: leaves through the lane's mailbox
  SQ_MBIN = 1 << 13,    // its parent: takes the next mailbox of the lane's source list
  SQ_FIRST = 1 << 14,   // first contribution into its slot: written, not added
  SQ_ROOT = 1 << 15,    // the cell root: no coupling to a parent
};
struct SeqLanes {
  bool built = false;
  int64_t nwaves = 0, nchunks = 0;
  int32_t max_slots = 0;            // most slots any lane uses
  int64_t depth_first = 0;          // lanes walked depth-first
  std::vector<KCellWave> waves;     // [nwaves], longest first
  std::vector<int32_t> lane_cell;   // [nwaves*64] cell of each lane, -1 for empty lanes
  std::vector<int64_t> base;        // [nwaves*64] first user index of the lane's cell (0: empty)
  std::vector<uint16_t> pos;        // [nchunks*kSeqChunkElems] staging order
  std::vector<uint16_t> code;       // [nchunks*kSeqChunkElems] cell-lane order
  std::vector<uint64_t> mbsrc;      // [nwaves*64] as CellLanes::mbsrc
};
// ERR_TOO_BIG if a cell has more than kCellMaxSize compartments or a lane
// needs more than kSeqSlots slots in both walk orders.
Status build_seq_lanes(const int32_t* parent, int64_t n, const int64_t* cell_offsets, int64_t ncells,
                       SeqLanes& out, std::string& err, int32_t cut_percent = 80,
                       int32_t max_cuts = kCellMaxCuts);
// Replay of the index-order tables: every compartment walked once, carries
// only from a child, every slot taken by a child of its owner, read by the
// owner and free again at the end, and each mailbox taken strictly after it
// was posted.
bool check_seq_lanes(const SeqLanes& Q, const int32_t* parent, int64_t n, const int64_t* cell_offsets,
                     int64_t ncells, std::string& why);

// LDS-resident solve (one wave per group of whole cells).  A group's d, u, b
// are staged into LDS once, as three planes in the user numbering (slot s
// holds user index lo + s; the planes are `stride` slots apart, a per-class
// constant that is a multiple of 64).  Each lane walks root-ward paths of the
// tree (paper §2: children before parents): a path starts at a leaf and
// follows parents up to its top, a compartment that is either a cell root or
// not the "heavy" child of its parent (the child whose subtree finishes last).
// A path is cut into chunks of kResK steps, padded at its bottom with steps on
// the zero entry (d = 1, u = 0, b = 0), so its top is the last step of its last
// chunk.  Inside a path the contribution to the next compartment stays in
// registers; a light path adds its top's contribution into its parent's LDS
// entry at the end of its last chunk, at least two chunks before the chunk
// that eliminates the parent (a lane reads a chunk's operands one chunk
// ahead).  The chunks are fixed at setup (an as-late-as-possible list schedule
// over the wave's 64 lanes); the forward sweep runs them in reverse.
constexpr int32_t kResK = 8;             // steps per chunk
constexpr int32_t kResEntBytes = 2 * kResK;  // slot-list entry: the byte offsets (uint16) of a chunk's steps
constexpr int32_t kResLaneTab = 272;     // 65 record offsets + 65 list offsets (uint16), padded
constexpr int32_t kResMaxSlots = 8000;   // image slots: 16-bit list entries hold slot * 8
constexpr int32_t kResNoParent = 0xffff; // record field: the top is a cell root
constexpr int32_t kResClasses = 10;
// LDS classes: class k holds floor(160 KiB / waves) bytes for waves = 1, 2, 3,
// 4, 5, 6, 7, 8, 10, 16 groups per CU; planes `stride` slots apart.
constexpr int32_t kResClassBytes[kResClasses] = {163840, 81920, 54528, 40960, 32768, 27136, 23296, 20480, 16384, 10240};
constexpr int32_t kResClassStride[kResClasses] = {6144, 3008, 1984, 1472, 1152, 960, 832, 704, 576, 320};
struct KResGroup {
  int64_t lo;          // user index of slot 0 (even)
  int64_t blob;        // first 16-byte unit of the group's blob
  int32_t nslot;       // slots of the image (even); slot nslot is the zero entry
  int32_t ndma;        // slots staged from the user arrays: min(nslot, n - lo)
  int32_t first;       // slot of the group's first compartment (0 or 1)
  int32_t count;       // compartments of the group
  int32_t nchunk;      // chunks per sweep
  int32_t blob_units;  // 16-byte units of the blob
  int32_t nroot;       // cells of the group
  int32_t npath;       // path records
  int32_t nlist;       // slot-list entries (one per active chunk of a lane)
  int32_t rec_off;     // byte offset of the records in the blob
  int32_t list_off;    // byte offset of the slot lists in the blob
  int32_t cls;         // LDS class (index into kResClassBytes / kResClassStride)
  int32_t nflip;       // couplings that move when the cells are re-rooted (pairs in the blob)
  int32_t pad;
};
static_assert(sizeof(KResGroup) == 72, "layout");
// Path record: first chunk, chunks, byte offset (slot * 8) of the top's parent
// entry or kResNoParent, spare.
struct KResRec {
  uint16_t c0, nch, par, spare;
};
static_assert(sizeof(KResRec) == 8, "layout");
// Blob of a group, in 16-byte units: per lane the first record and the first
// slot-list entry (65 + 65 uint16, kResLaneTab bytes), the root slots of its
// cells (uint16, padded to 16 bytes), the re-rooting pairs (uint16 slot whose
// coupling to its new parent is the u staged at the second uint16 slot; padded
// to 16 bytes), the records lane by lane in chunk order,
// then the slot lists: per lane, one kResEntBytes entry per active chunk, in
// chunk order, holding the byte offsets (slot * 8) of the chunk's kResK steps from
// the bottom of the path upward.
constexpr int64_t res_lds_bytes(int32_t cls, int64_t blob_units) {
  return 24 * (int64_t)kResClassStride[cls] + 16 * blob_units;
}
// Target of the packing: consecutive cells share a group while it holds at
// most this many compartments (a larger cell is a group of its own).
constexpr int32_t kResPackSlots = 1400;

struct ResPlan {
  bool built = false;
  std::vector<KResGroup> groups;
  std::vector<uint8_t> blob;   // group blobs, 16-byte aligned
  int64_t max_lds = 0;
};

// Build the LDS-resident tables; parent / cell_offsets must already be valid.
// ERR_TOO_BIG if a cell's image does not fit the largest LDS class.
// pack: consecutive cells share a group while it holds at most this many
// compartments (kResPackSlots by default).
Status build_resident(const int32_t* parent, int64_t n, const int64_t* cell_offsets, int64_t ncells,
                      ResPlan& out, std::string& err, int32_t pack = kResPackSlots, bool reroot = false);
// Replay of the resident tables: every record, list entry and slot inside its
// group image, every compartment eliminated once, after all its children, and
// every light path's contribution added two chunks before its parent's chunk.
bool check_resident(const ResPlan& R, const int32_t* parent, int64_t n, std::string& why);

// Per-branch record of the LDS-staged solve kernel, in (group, level, lane)
// order; 16 bytes so that one DMA lane moves one record.  All indices are
// group-local: positions in the group's LDS image (its cells concatenated in
// packing order) or group-local breadth-first branch ids.  A group's LDS image
// holds at most a few thousand compartments, far inside int16.
struct KBranch {
  int16_t start;   // LDS index of the branch's root-side compartment
  int16_t lendir;  // len, negated when the branch runs toward lower user indices
  int16_t u0;      // LDS index of the coupling of position 0 to its parent (-1: root)
  int16_t pslot;   // LDS index of the parent compartment (-1: root)
  int16_t self;    // group-local breadth-first id (slot of its elimination contribution)
  int16_t child0;  // group-local id of the first child branch
  int16_t nchild;  // number of child branches (ids child0 .. child0+nchild-1)
  int16_t pad;     // unused (0)
};
static_assert(sizeof(KBranch) == 16, "one DMA lane per record");

constexpr int32_t kMaxGroupSlots = 32766;  // largest LDS image the int16 records address
// Unused slots in front of and behind a group's compartments in its LDS image,
// so that the solve kernels may read a fixed window of 8 compartments around
// any position without bounds checks.
constexpr int32_t kLdsPad = 8;

struct KGroup {
  int64_t user_base;   // contiguous groups: user index of LDS slot kLdsPad (even)
  int64_t ws_off;      // groups whose image exceeds LDS: offset (doubles) of the image in the
                       // global workspace; -1 for groups staged in LDS
  int32_t seg_begin;   // first entry of this group in the segment table
  int32_t nlev;        // levels (segments)
  int32_t cell_begin;  // first entry in the group-cell table
  int32_t ncell;
  int32_t nunk;        // LDS slots per array: compartments + alignment padding (even)
  int32_t nbr;         // branches in the group
  int32_t cost;        // sum over levels of the longest branch (critical path)
  int32_t br_begin;    // first record of the group in the branch table
  int32_t contig;      // 1: cells are one user range; LDS slot kLdsPad + k <-> user index user_base + k
  int32_t user_lo;     // contiguous groups: first user index relative to user_base (0 or 1)
  int32_t user_n;      // contiguous groups: compartments in the range
  int32_t makespan;    // flow kernel: steps of each sweep (0: not scheduled)
};
static_assert(sizeof(KGroup) == 64, "layout");

struct KCell {
  int64_t user_lo;  // first user index of the cell
  int32_t n;        // compartments
  int32_t lds;      // offset of the cell in the group's LDS image
};

// Flow kernel tables of one group.  The compartments (and path pads) get LDS
// "entries" in chunk-step order: the chunk of lane l at chunk step t is block
// R[t] + (active lanes below l at t), R[t] the active lane-chunks before t,
// and sub-step j is entry j of that block.  Entries are named by their LDS
// offset in 8-byte units (block * kFlowBlock8 + 3 j).  Per chunk step the
// table holds two 64-bit lane masks (active; push: the lane ends a path whose
// contribution goes to LDS); per element of the group's staging order its
// entry (bit 15: the cell root, whose coupling is ignored); per push, in
// (step, lane) order, the entry of the parent compartment.
struct KFlow {
  int64_t step_off;  // first step record (two uint64 masks) of the group
  int64_t pos_off;   // first element entry
  int64_t aux_off;   // first push target
  int32_t nstep;     // chunk steps per sweep (0: not a flow group)
  int32_t nelem;     // compartments
  int32_t naux;      // pushes
  int32_t makespan;  // chunk steps
  int32_t nent;      // entries: compartments and pads (kFlowChunk per block)
  int32_t pad1;
};
static_assert(sizeof(KFlow) == 48, "layout");

// LDS layout of a flow group: image (24 bytes per entry: d, u, b; then one
// constant entry for idle lanes and 64 write-only sink entries), push targets
// (int16, at least one entry), step masks (16 bytes per step plus a zero
// record before and after).
constexpr int64_t flow_image8(const KFlow& w) {  // 8-byte units of blocks, identity block and sink
  return (int64_t)w.nent / kFlowChunk * kFlowBlock8 + kFlowTail8;
}
constexpr int64_t flow_mask_offset(const KFlow& w) {
  return (8 * flow_image8(w) + 2 * ((int64_t)w.naux + 1) + 15) & ~(int64_t)15;
}
constexpr int64_t flow_lds_bytes(const KFlow& w) { return flow_mask_offset(w) + 16 * ((int64_t)w.nstep + 2); }

struct HostPlan {
  int64_t n = 0, ncells = 0, nbranches = 0, ngroups = 0, nseg = 0;
  int32_t max_level = -1;
  Options opt;

  // exported tables (compact)
  std::vector<int32_t> node_plan;                       // [n]
  std::vector<int32_t> br_cell, br_level, br_first, br_dir, br_len, br_parent, br_group, br_rank;
  std::vector<int32_t> u_src;                           // [n], plan order
  std::vector<int64_t> group_offsets, group_cells, group_seg_offsets, seg_offsets;
  std::vector<int32_t> lanes;                           // [nb]

  // kernel tables
  std::vector<KBranch> kbranch;   // [nb] lane order
  std::vector<KGroup> kgroup;     // [ngroups]
  std::vector<int32_t> kseg;      // [nseg+1] begin of each segment in kbranch
  std::vector<KCell> kcell;       // [ncells] group order
  bool kernel_tables_fit = true;  // every group addressable by the int16 records
  bool all_ascending = true;      // every branch runs toward higher user indices
  bool flow = false;              // every LDS group has a step schedule (flow kernel)
  std::vector<KFlow> kflow;       // [ngroups]
  std::vector<uint64_t> fmask;    // [2 * total steps]: active and push masks per step
  std::vector<uint16_t> fpos;     // [elements of LDS groups]: position, bit 15 = cell root
  std::vector<int16_t> faux;      // [pushes]: parent position
  int64_t ws_doubles = 0;         // global workspace for groups that exceed LDS
  CellLanes cl;                   // cell-lane kernel tables (opt.cell_lanes)
  SeqLanes sq;                    // index-order cell-lane tables (opt.cell_seq)
  ResPlan res;                    // LDS-resident kernel tables (opt.resident)
};

Status build_plan(const int32_t* parent, int64_t n, const int64_t* branch_offsets, int64_t nbranches,
                  const int64_t* cell_offsets, int64_t ncells, const Options& opt, HostPlan& out,
                  std::string& err);

// Copy table `id` into out (int64), returns the element count (or -1).
int64_t export_table(const HostPlan& p, int32_t id, int64_t* out, int64_t capacity);

}  // namespace hines
