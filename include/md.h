/*
 * md.h -- C ABI of libmd, an MI355X (gfx950) library for the hot path of
 * short-range non-bonded molecular dynamics as studied in arXiv 2109.10876
 * ("Code modernization strategies for short-range non-bonded molecular
 * dynamics simulations"): Lennard-Jones pair forces with a cutoff, evaluated
 * over cell-list-built Verlet neighbour lists with a skin, on a
 * structure-of-arrays particle layout, inside a velocity-Verlet step.
 *
 * General rules for every call below
 * ----------------------------------
 *  - Pointers named in structs or arguments are DEVICE pointers unless the
 *    argument name starts with h_ (host).  The caller allocates and owns every
 *    buffer; the library keeps no pointer between calls and never allocates.
 *  - Work is only enqueued on `stream` (a hipStream_t passed as void*; NULL is
 *    the null stream).  No call synchronises, so every call may be captured in
 *    a HIP graph.  Calls that share a workspace must be ordered (same stream).
 *  - Host-detectable errors are returned immediately (negative MD_E* code)
 *    and nothing is enqueued.  Errors found on the device are sticky bits
 *    OR-ed into *status (MD_F_*); the caller clears the word and reads it
 *    after synchronising.  Nothing is ever truncated silently.
 *  - Batching: a call works on R independent replicas ("systems") at once.
 *    Replica r owns atoms [atom_off[r], atom_off[r+1]) and cells
 *    [cell_off[r], cell_off[r+1]).  R = 1 is the single-system case.
 *  - Per-atom arrays are structure-of-arrays planes (Sec. 3.1 of the paper:
 *    each attribute in its own array).  After md_cell_sort they are in cell
 *    order; `id` keeps each atom's original global index.
 *  - gate (optional, [R] uint32): replicas with gate[r] == 0 are skipped by
 *    md_cell_sort and md_verlet_build.  NULL means "all replicas".
 */
#ifndef MD_H
#define MD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MD_ABI_VERSION 11

/* ------------------------------------------------------------ return codes */
#define MD_OK            0
#define MD_EINVAL       -1  /* null/misaligned pointer, bad count, mode or precision   */
#define MD_EBOX         -2  /* a box edge < 2 (rc + skin): minimum image not unique    */
#define MD_ENOWS        -3  /* workspace smaller than md_workspace_bytes()             */
#define MD_EUNSUPPORTED -4  /* valid request this build does not implement             */
#define MD_EHIP         -5  /* a HIP launch failed                                     */
#define MD_ERANGE       -6  /* sizes beyond the encoding limits below                  */
#define MD_ESCRATCH     -7  /* batch needs more than MD_NOALLOC_SCRATCH_BYTES          */

/* ------------------------------------------------ device status bits (sticky) */
#define MD_F_NBR_OVERFLOW 0x1u  /* some atom has more list entries than max_nbr     */
#define MD_F_NONFINITE    0x2u  /* a force or energy came out NaN/Inf               */
#define MD_F_BOND_BROKEN  0x4u  /* a FENE bond reached its maximum extension        */
#define MD_F_TILE_OVERFLOW 0x8u /* a tile's staged neighbourhood exceeds MD_TILE_SLOTS */

/* ------------------------------------------------------------------- enums */
#define MD_HALF 0         /* each unordered pair stored once (Newton's third law) */
#define MD_FULL 1         /* each pair stored for both atoms                      */
#define MD_TILE_FULL 2    /* full list in tile-local form (see "Tile-local lists")  */
#define MD_BY_ID 0        /* bonded table keyed by atom id, naming atom ids        */
#define MD_BY_INDEX 1     /* bonded table keyed by current index, naming indices   */
#define MD_FP64 0         /* all pair arithmetic in double precision              */
#define MD_FP32_MIXED 1   /* distances, cutoff test and force accumulation in
                             double; reciprocal and LJ polynomial in single     */

/* ------------------------------------------------------------------ limits */
#define MD_UNIT_ATOMS 256           /* atoms per work unit (one workgroup)        */
#define MD_IDX_BITS   26            /* list entry: low 26 bits = neighbour index  */
#define MD_IDX_MASK   0x03FFFFFFu
#define MD_MAX_ATOMS  0x03FFFFFF    /* total atoms per call                       */
#define MD_MAX_TYPES  8             /* atom types                                 */
#define MD_MAX_BONDS  4             /* bonds per atom                             */
#define MD_MAX_ANGLES 8             /* angle triples an atom belongs to           */
#define MD_TILE_SLOTS 3072          /* staged atoms per tile (MD_TILE_FULL)       */
#define MD_TILE_MAX_CELLS 64        /* cells per tile along x                     */
#define MD_TILE_MAX_ROWS  2         /* cell rows per tile along y and along z     */
#define MD_TILE_MAX_TYPES 4         /* atom types of a typed tile-local list      */

/* Verlet-list entry encoding.  Entry e of atom i names atom j = e & MD_IDX_MASK
 * and the periodic image under which j is i's neighbour: for dimension d
 * (x, y, z), the two bits (e >> (26 + 2d)) & 3 hold s_d = 0, +1 (code 1) or
 * -1 (code 2), and the minimum-image displacement is
 *     d_d = x_i[d] - x_j[d] + s_d * L_d.
 * The image is fixed when the list is built and stays valid until the next
 * rebuild because positions are only wrapped into the box at rebuild time. */

/* Tile-local lists (mode MD_TILE_FULL).  The cells of each replica are cut
 * into tiles of tile_cells x tile_py x tile_pz cells along x, y, z (tiles at
 * the high end of a dimension may be smaller), numbered replica by replica,
 * then z-block, y-block, x-block (x fastest).  For a tile with home cells
 * x in a..b, y in y0..y1, z in z0..z1, the staged neighbourhood is, for z
 * from z0-1 to z1+1 and within it y from y0-1 to y1+1 (each wrapped
 * periodically with the image the wrap implies), the cells of unwrapped
 * x = a-1 .. b+1 of that row (x = -1 is cell nx-1 one box length to the
 * left, x = nx is cell 0 one box length to the right), each cell's atoms in
 * index order, concatenated.  Entries come in blocks of 8 per atom: entry k
 * of atom i is the uint16 ((uint16_t *)idx)[(k / 8) * 8 ld + 8 i + k % 8]
 * = 8 p + t, where p is the position of the neighbour in its tile's staged
 * sequence (its image is the one its staged row and cell imply) and t is its
 * atom type when tile_types > 1 (else 0).  Entries count[i] .. (count[i]
 * rounded up to 16) - 1 hold 8 md_tile_capacity(), a pad slot far from every
 * atom, so max_nbr must be a multiple of 16, ld at most 2^23 and idx
 * 16-byte aligned (MD_EINVAL otherwise).  Pairs are those within rc + skin up to rounding: the tile
 * build may keep a pair whose distance exceeds rc + skin by rounding only.
 * A tile whose staged
 * sequence exceeds md_tile_capacity() (at most MD_TILE_SLOTS) raises
 * MD_F_TILE_OVERFLOW (the list is then unusable: rebuild with smaller
 * tiles).  md_lj_forces and md_lj_forces_vjp take a tile-local list whose
 * tile_types equals the LJ table's ntypes (0 or 1 for one type), at most
 * MD_TILE_MAX_TYPES (MD_EINVAL / MD_EUNSUPPORTED otherwise). */

/* ------------------------------------------------------------------ structs */

/* Partition of the atoms into replicas, cells and work units.  Fill the
 * host-side arrays with md_plan_fill() and copy them to the device. */
typedef struct md_batch {
    int32_t R;                /* replicas, >= 1                                  */
    int32_t N;                /* total atoms, 1 .. MD_MAX_ATOMS                  */
    int32_t C;                /* total cells                                     */
    int32_t n_units;          /* work units: ceil(N_r / MD_UNIT_ATOMS) summed    */
    const int32_t *atom_off;  /* [R+1] first atom of each replica                */
    const int32_t *cell_off;  /* [R+1] first cell of each replica                */
    const int32_t *ncell;     /* [3R] cells per dimension (x, y, z)              */
    const double  *box;       /* [3R] orthorhombic box edges L_x, L_y, L_z       */
    const int32_t *unit_rep;  /* [n_units] replica of each work unit             */
    const int32_t *unit_off;  /* [R+1] first work unit of each replica           */
} md_batch;

/* Structure-of-arrays atom state, N entries per plane (img: 3 planes of N). */
typedef struct md_atoms {
    double  *x, *y, *z;       /* positions                                        */
    double  *vx, *vy, *vz;    /* velocities                                       */
    double  *fx, *fy, *fz;    /* forces                                           */
    double  *xb, *yb, *zb;    /* positions at the last list build                 */
    int32_t *type;            /* atom type in [0, ntypes)                         */
    int32_t *id;              /* original global index, unique in [0, N)          */
    int32_t *img;             /* [3N] periodic image counters, planes x | y | z   */
    int32_t *where;           /* optional [N]: where[id] = current index          */
    double  *pos4;            /* optional [4N] packed (x, y, z, 0) per atom: when
                                 set, md_cell_sort and md_vv_step keep it equal to
                                 the x, y, z planes and the pair kernels gather
                                 neighbour positions from it (one 32-byte load
                                 instead of three 8-byte loads from three planes) */
} md_atoms;

/* Verlet list in ELL layout, column-major so that entry k of consecutive
 * atoms is contiguous: entry k of atom i is idx[k * ld + i] (MD_TILE_FULL:
 * uint16 entries in blocks of 8, see "Tile-local lists"). */
typedef struct md_nlist {
    int32_t  mode;            /* MD_HALF, MD_FULL or MD_TILE_FULL                 */
    int32_t  max_nbr;         /* capacity per atom (columns)                      */
    int32_t  ld;              /* leading dimension, >= N and a multiple of 64     */
    int32_t  tile_cells;      /* MD_TILE_FULL: cells per tile, 1..md_tile_max_cells() */
    int32_t  *count;          /* [N] true entry count (may exceed max_nbr)        */
    uint32_t *idx;            /* [max_nbr * ld] uint32 entries; MD_TILE_FULL uses
                                 the first half as [max_nbr * ld] uint16 entries  */
    int32_t  n_tiles;         /* MD_TILE_FULL: tiles (md_tile_plan)               */
    int32_t  tile_py;         /* MD_TILE_FULL: cell rows per tile along y, 1..2   */
    int32_t  tile_pz;         /* MD_TILE_FULL: cell rows per tile along z, 1..2   */
    int32_t  tile_types;      /* MD_TILE_FULL: 0 or 1 = entries carry no type;
                                 2..MD_TILE_MAX_TYPES = entries carry the
                                 neighbour's type (set to the LJ table's ntypes) */
    const int32_t *tile_rep;  /* MD_TILE_FULL: [n_tiles] replica of each tile     */
    const int32_t *tile_off;  /* MD_TILE_FULL: [R+1] first tile of each replica   */
    int32_t  *tile_need;      /* optional: largest staged count seen (overflow)   */
    const int32_t *cell_start;/* MD_TILE_FULL: the [C+1] cell ranges the list was
                                 built with (unchanged until the next rebuild)    */
    int32_t  tile_src_cap;    /* MD_TILE_FULL: the md_tile_capacity() tile_src was
                                 sized for; calls whose current capacity differs
                                 return MD_EINVAL                              */
    int32_t  _pad;
    uint32_t *tile_src;       /* MD_TILE_FULL: [n_tiles * (tile_src_cap + 128)]
                                 staging record of every tile (each staged slot's
                                 source atom and image), written by
                                 md_verlet_build and read by md_lj_forces,
                                 md_lj_forces_vv and md_lj_forces_vjp (which also
                                 keeps per-tile sums in it); part of the list  */
    int32_t *tile_active;     /* MD_TILE_FULL, optional, one replica only:
                                 [2 n_tiles + 1], zero-filled before the first
                                 build.  md_verlet_build lists the tiles that
                                 have home atoms: tile_active[0] = their count,
                                 tile_active[1 ..] the tiles in ascending order
                                 (the rest is its bookkeeping).  md_lj_forces
                                 and md_lj_forces_vv then give workgroups to
                                 listed tiles only, so the vacuum of a sparse
                                 system costs no staging.  NULL: every tile. */
    const int32_t *tile_m;    /* MD_TILE_FULL, optional: [R] device, replica r's
                                 cells per tile along x (1 .. tile_cells), the
                                 h_tile_m the tiles were planned with, so that
                                 each replica takes the largest tiles its own
                                 cell occupancy fits.  NULL: tile_cells for
                                 every replica.                                */
    int32_t *tile_todo;       /* MD_TILE_FULL, optional: [n_tiles + 1] device
                                 scratch of md_verlet_build on a batch (R > 1)
                                 called with a gate: it first lists the tiles
                                 of the replicas to rebuild there (their count,
                                 then the tiles), so that a workgroup per
                                 listed tile builds and every other one returns
                                 after one load.  NULL: each tile reads its
                                 replica's gate.                               */
} md_nlist;

/* Lennard-Jones parameters (Eq. lj: U = 4 eps [(sig/r)^12 - (sig/r)^6] for
 * r < rc), per type pair, in symmetric [ntypes * ntypes] row-major tables. */
typedef struct md_lj {
    int32_t ntypes;           /* 1 .. MD_MAX_TYPES                                */
    int32_t shift;            /* 1: energy lowered by U(rc) (continuous at rc)    */
    double  rc;               /* cutoff radius                                    */
    const double *eps;        /* [ntypes*ntypes] device                           */
    const double *sig;        /* [ntypes*ntypes] device                           */
} md_lj;

/* Bonds, indexed by original atom id (stable across re-sorts): partner k of
 * the atom whose id is a is partner[k * N + a] (an id), k < count[a].  Each
 * bond is listed for both of its atoms. */
/* Bonds, stored for both of their atoms.  With order MD_BY_ID, column a
 * belongs to the atom with id a and partner entries are atom ids in [0, N);
 * with MD_BY_INDEX (written by md_bonded_reindex), column i belongs to the
 * atom now at index i and entries are current indices, valid until the next
 * md_cell_sort moves atoms. */
typedef struct md_bonds {
    int32_t max_bonds;        /* columns of partner, 1 .. MD_MAX_BONDS            */
    int32_t order;            /* MD_BY_ID or MD_BY_INDEX                          */
    const int32_t *count;     /* [N] bonds of atom a                              */
    const int32_t *partner;   /* [max_bonds * N] partners, slot k at k N + a      */
} md_bonds;

/* Angle triples (a, b, c), b the middle bead, stored once per member atom so
 * that each atom can sum its own share: slot k (< count[a]) of atom a names
 * the triple (tri[(3k) N + a], tri[(3k+1) N + a], tri[(3k+2) N + a]), and
 * atom a is one of the three.  A triple names three distinct atoms.  Keys and
 * entries are ids or current indices as for md_bonds. */
typedef struct md_angles {
    int32_t max_angles;       /* slots per atom, 1 .. MD_MAX_ANGLES                */
    int32_t order;            /* MD_BY_ID or MD_BY_INDEX                           */
    const int32_t *count;     /* [N] triples of atom a                             */
    const int32_t *tri;       /* [3 * max_angles * N] members, by slot and role    */
} md_angles;

/* Langevin thermostat of md_lj_forces_vv: the force of md_langevin (same
 * normals, same counter) with these parameters. */
typedef struct md_thermostat {
    double gamma;             /* friction, >= 0                                   */
    double temperature;       /* target T, >= 0                                   */
    uint64_t seed;            /* Philox key                                       */
    uint64_t *step;           /* device, one uint64: the noise counter, read by
                                 every atom and then advanced by one            */
    const double *mass;       /* [ntypes] device: m of each type                  */
} md_thermostat;

/* ---------------------------------------------------------------- plumbing */

int         md_abi_version(void);
const char *md_strerror(int code);

/* Process-wide tuning knobs, read on the host at launch time.  They change
 * speed only, never results beyond summation order (FP64 paths stay
 * bitwise deterministic for a fixed setting).  md_tune_set returns
 * MD_EINVAL for an unknown knob or value. */
#define MD_TUNE_PAIR_BATCH 0   /* list entries whose neighbour positions are
                                  gathered together in the force and VJP loops:
                                  1, 2, 4 or 8 (default 4)                      */
#define MD_TUNE_TILE_THREADS 1 /* workgroup size of the tile-local kernels: 64, 128
                                  or 256 (default 256); staged capacity 1024, 1792
                                  or 3072 atoms (md_tile_capacity).  Change it only
                                  before a rebuild of MD_TILE_FULL lists.        */
#define MD_TUNE_TILE_STAGE_PACKED 2 /* 1: tile staging reads the packed copy when
                                  present; 0 (default): the x, y, z planes      */
#define MD_TUNE_TILE_SLOTS 3   /* staged capacity of the 256-thread tile shape:
                                  0 (default) or 3072 (up to 64 cells per tile),
                                  2048 (16 cells) or 1536 (8 cells).  Less LDS
                                  per workgroup lets more of them share a CU
                                  (force kernels: two, three and four).
                                  Change it only before a rebuild of
                                  MD_TILE_FULL lists.                           */
#define MD_TUNE_NKNOBS     4
int md_tune_set(int32_t knob, int32_t value);
int md_tune_get(int32_t knob);
/* Measurement aid.  md_kernel_timing_start(n) (0 <= n <= 1024) has the next
 * n pair-force kernel launches of md_lj_forces and md_lj_forces_vv that are
 * not under stream capture record a HIP event pair around the kernel alone,
 * on the launch's stream; md_kernel_timing_read waits for the recorded pairs
 * and gives their mean duration in ms and their count.  Process-wide state,
 * not thread-safe; MD_EINVAL for n out of range or null outputs, MD_EHIP if
 * an event cannot be read. */
int md_kernel_timing_start(int32_t n);
int md_kernel_timing_read(double *mean_ms, int32_t *count);
/* Measurement aid: copies `bytes` bytes from device buffer src to device
 * buffer dst (caller-owned, 16-byte aligned, not overlapping) with a plain
 * streaming kernel on `stream` (a hipStream_t).  Timing it gives the HBM
 * bandwidth a kernel can reach (bytes read + bytes written over the
 * duration), the denominator of the roofline fraction, and it is the
 * known-size kernel that calibrates the HBM byte counters.  MD_EINVAL for null
 * or misaligned pointers or a size that is 0 or not a multiple of 16,
 * MD_ERANGE for sizes beyond 2^31 blocks of 16 KiB, MD_EHIP on a launch
 * failure. */
int md_copy_probe(const void *src, void *dst, size_t bytes, void *stream);
/* Staged-atom capacity per tile of MD_TILE_FULL lists for the current
 * MD_TUNE_TILE_THREADS and MD_TUNE_TILE_SLOTS (a tile whose staged sequence
 * is larger raises MD_F_TILE_OVERFLOW). */
int md_tile_capacity(void);
/* Largest tile_cells the current tile shape accepts (a list with more makes
 * md_verlet_build and md_lj_forces return MD_EINVAL). */
int md_tile_max_cells(void);

/* Host-only planning (no GPU work).  Cells per dimension n_d = floor(L_d /
 * (rc + skin)) so that the cell edge is at least rc + skin (Sec. 2.1.2).
 * Returns MD_EBOX if some L_d < 2 (rc + skin), MD_EINVAL for R < 1, an empty
 * replica or non-positive radii, MD_ERANGE if sizes exceed the limits. */
int md_plan_sizes(int32_t R, const int32_t *h_natoms, const double *h_box,
                  double rc, double skin,
                  int32_t *h_N, int32_t *h_C, int32_t *h_n_units);
/* Fills atom_off[R+1], cell_off[R+1], ncell[3R], unit_rep[n_units] and
 * unit_off[R+1] (host arrays sized from md_plan_sizes). */
int md_plan_fill(int32_t R, const int32_t *h_natoms, const double *h_box,
                 double rc, double skin,
                 int32_t *h_atom_off, int32_t *h_cell_off, int32_t *h_ncell,
                 int32_t *h_unit_rep, int32_t *h_unit_off);

/* Tiles of MD_TILE_FULL lists: with h_tile_rep/h_tile_off NULL returns the
 * number of tiles of m_r x tile_py x tile_pz cells (h_ncell as from
 * md_plan_fill), m_r = h_tile_m[r] (optional [R] host array, each in
 * 1 .. tile_cells) or tile_cells for every replica when h_tile_m is NULL;
 * otherwise also fills h_tile_rep[n_tiles] and h_tile_off[R+1].  Negative
 * MD_E* on bad arguments. */
int md_tile_plan(int32_t R, const int32_t *h_ncell, int32_t tile_cells,
                 const int32_t *h_tile_m, int32_t tile_py, int32_t tile_pz,
                 int32_t *h_tile_rep, int32_t *h_tile_off);

/* Bytes of the device workspace used by the calls below for this batch.
 * The workspace must be zero-filled once after allocation; every call
 * leaves the parts that must start at zero back at zero. */
size_t md_workspace_bytes(const md_batch *b);

/* ------------------------------------------------------------- the path */

/* Cell binning and re-sort ("Resort", Sec. 2.1.3 and Sec. 3.1): wraps
 * positions into the box (updating img), bins atoms into cells, orders atoms
 * cell by cell (ascending id inside a cell, so the order is deterministic),
 * permutes x, v, type, id, img of `atoms` in place (through `scratch`, whose
 * x, y, z, vx, vy, vz, type, id, img planes must be distinct N-sized
 * buffers), sets x_build := x, fills cell_start[C+1] (cell c holds atoms
 * [cell_start[c], cell_start[c+1])) and, if atoms->where is set, where[].
 * Forces are not carried through the permutation.  Replicas whose gate is
 * zero are left untouched. */
int md_cell_sort(const md_batch *b, md_atoms *atoms, md_atoms *scratch,
                 int32_t *cell_start, void *ws, size_t ws_bytes,
                 const uint32_t *gate, uint32_t *status, void *stream);

/* Verlet list build (Sec. 2.1.2, Sec. 3.2 "SortedList"): for each atom, the
 * atoms of its own cell and the 26 neighbouring cells (each distinct cell
 * once) whose minimum-image distance is < rc + skin.  MD_FULL lists every
 * neighbour; MD_HALF lists pair (i, j) only at i < j.  The per-atom order is
 * cells in (z, y, x) stencil order, then ascending index -- deterministic.
 * If an atom has more than max_nbr entries its count still holds the true
 * number, MD_F_NBR_OVERFLOW is raised and *need (device int32, optional)
 * receives the maximum count; the list is then unusable until rebuilt with
 * max_nbr >= need.  Expects atoms sorted by md_cell_sort.  For MD_TILE_FULL
 * lists it also writes each tile's staging table (nl->tile_src), which the
 * force calls read instead of re-deriving the staged sequence. */
int md_verlet_build(const md_batch *b, const md_atoms *atoms,
                    const int32_t *cell_start, double rc, double skin,
                    md_nlist *nl, int32_t *need, const uint32_t *gate,
                    uint32_t *status, void *stream);

/* Lennard-Jones forces, potential energy and virial (Eq. lj) over the list:
 * F_i = sum_j fr(r_ij) d_ij with fr = -U'(r)/r for r < rc, E_r = sum over
 * pairs of U (minus U(rc) if shift), W_r = sum over pairs of fr r^2.
 * accumulate = 0 overwrites fx, fy, fz; 1 adds to them.  energy/virial ([R],
 * optional) receive per-replica totals, reduced in a fixed order (FP64).
 * MD_FULL results are bitwise deterministic; MD_HALF uses atomic adds for
 * the partner atom's force.  prec = MD_FP64 or MD_FP32_MIXED. */
int md_lj_forces(const md_batch *b, const md_atoms *atoms, const md_nlist *nl,
                 const md_lj *p, int32_t prec, int32_t accumulate,
                 double *energy, double *virial, void *ws, size_t ws_bytes,
                 uint32_t *status, void *stream);

/* md_lj_forces without a workspace argument, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc.  Arguments, results, errors and
 * determinism are those of md_lj_forces (the same kernels, bit for bit).  The
 * scratch the call needs -- per-work-unit partial sums (n_units rows of 32
 * bytes) and, for MD_TILE_FULL lists, per-tile partial sums (n_tiles rows of
 * 32 bytes) -- lives in a fixed array of MD_NOALLOC_SCRATCH_BYTES inside the
 * library, one per GPU, held from the first call on that GPU until the
 * process ends.  That first call looks the array up on the current device
 * (the stream must belong to it); no call allocates.  A batch needing more
 * returns MD_ESCRATCH before anything is enqueued.  Every call on one GPU
 * shares its array: calls that may overlap on one GPU (different streams,
 * or threads) race and must be serialised by the caller. */
#define MD_NOALLOC_SCRATCH_BYTES (8u << 20)
int md_lj_forces_noalloc(const md_batch *b, const md_atoms *atoms, const md_nlist *nl,
                         const md_lj *p, int32_t prec, int32_t accumulate, double *energy,
                         double *virial, uint32_t *status, void *stream);

/* md_lj_forces followed, in the same kernel, by md_vv_step phase 3 for each
 * atom as soon as its force is known (the forces of a step feed its
 * Integrate2 and the next step's Integrate1 directly): on return fx, fy, fz
 * hold the forces at the positions on entry, velocities and positions are
 * advanced, gate[r] and ke[r] (optional) are set as by md_vv_step phase 3,
 * energy/virial as by md_lj_forces.  Pair forces over MD_TILE_FULL lists
 * (MD_EUNSUPPORTED otherwise; with several atom types, up to
 * MD_TILE_MAX_TYPES, over a typed list as md_lj_forces needs), optionally with the
 * Langevin thermostat: with thermo set, each atom's force also receives the
 * md_langevin force (velocity on entry, noise counter *thermo->step, which
 * is then advanced by one) before the integrator uses it, as md_lj_forces,
 * md_langevin and md_vv_step phase 3 in sequence would.  A step that adds
 * bond forces uses the separate calls.  The same arithmetic as those calls
 * in sequence, so trajectories agree to rounding of the thermostat sum (and
 * bitwise without it); the kinetic energy is summed in another order.  New positions:
 * with x_next, y_next, z_next NULL they are staged in the workspace and
 * copied back into atoms->x, y, z (and the packed copy, if set); with all
 * three given ([N] device each, not overlapping atoms->x, y, z; atoms->pos4
 * must be NULL) they are written there and atoms->x, y, z stay as they were,
 * so a caller that alternates two position buffers skips the copy.  Other
 * combinations return MD_EINVAL.  gate_clear (optional, [R] device, not
 * overlapping gate, not with thermo): the call then zeroes gate_clear and sets
 * gate[r] to 1 if an atom of replica r moved more than skin/2, leaving it as
 * it is otherwise (with one atom type from the force kernel itself, so that
 * no finaliser runs when ke, energy and virial are NULL; with several, from
 * the finaliser); a caller that passes two words alternately, each the
 * gate of one call and the gate_clear of the next, gets the gate of
 * md_vv_step phase 3 on every call once both start at zero. */
int md_lj_forces_vv(const md_batch *b, md_atoms *atoms, const md_nlist *nl, const md_lj *p,
                    int32_t prec, double dt, const double *inv_mass, int32_t ntypes,
                    double skin, uint32_t *gate, uint32_t *gate_clear, double *ke,
                    double *energy, double *virial,
                    double *x_next, double *y_next, double *z_next,
                    const md_thermostat *thermo, void *ws, size_t ws_bytes,
                    uint32_t *status, void *stream);

/* Velocity-Verlet update (Sec. 2.1, Fig. 1: Integrate1 / Integrate2).
 *  phase 1: v += dt/2 F/m; x += dt v; gate[r] = 1 if some atom of replica r
 *           moved more than skin/2 from x_build (the list may miss a pair
 *           within rc), else 0.
 *  phase 2: v += dt/2 F/m; ke[r] = sum 1/2 m v^2.
 *  phase 3: phase 2 immediately followed by phase 1 in one pass (ke is taken
 *           between the two half kicks).
 * inv_mass: [ntypes] device array of 1/m.  gate is required for phases 1 and
 * 3; ke is optional.  thermo (optional, phases 2 and 3 only, MD_EINVAL for
 * phase 1): before its half kick each atom adds the md_langevin force, with
 * the velocity on entry and noise counter *thermo->step (then advanced by
 * one), to fx, fy, fz, so that the calls md_langevin then md_vv_step become
 * one pass (the forces were evaluated at that velocity). */
int md_vv_step(const md_batch *b, md_atoms *atoms, int32_t phase, double dt,
               const double *inv_mass, int32_t ntypes, double skin,
               uint32_t *gate, double *ke, const md_thermostat *thermo, void *ws,
               size_t ws_bytes, uint32_t *status, void *stream);

/* Vector-Jacobian product of md_lj_forces (the derivatives of Eq. lj's pair
 * force and energy, Sec. 2.1.1, with respect to positions, eps and sigma):
 * given G = dL/dF (planes gfx, gfy, gfz, [N] each, same atom order) and gE
 * ([R], dL/dE_r, optional), writes gx = dL/dx (planes [3N]) and, optionally,
 * geps and gsig ([ntypes^2], derivatives with respect to the shared parameter
 * of each unordered type pair; both mirrored entries hold it, summed over all
 * replicas).  Pair terms are recomputed from the list, nothing is stored by
 * md_lj_forces.  Requires an MD_FULL list or an MD_TILE_FULL list (at most
 * MD_TILE_MAX_TYPES types, typed as for md_lj_forces; MD_EUNSUPPORTED for
 * MD_HALF).  prec = MD_FP32_MIXED on a tile list evaluates each pair term in
 * single precision (G rounded to it) and sums in double. */
int md_lj_forces_vjp(const md_batch *b, const md_atoms *atoms, const md_nlist *nl,
                     const md_lj *p, int32_t prec, const double *gfx,
                     const double *gfy, const double *gfz, const double *gE,
                     double *gx, double *geps, double *gsig, void *ws,
                     size_t ws_bytes, uint32_t *status, void *stream);

/* FENE bonds of the bead-spring polymer melt (Sec. 4 of the paper, after
 * Kremer and Grest): U(r) = -(1/2) K R0^2 ln(1 - r^2/R0^2) with force factor
 * fr = -K / (1 - r^2/R0^2), minimum-image bond vector.  Forces are ADDED to
 * fx, fy, fz (call after md_lj_forces).  A table keyed by id needs
 * atoms->where (id -> current index, kept by md_cell_sort); a table keyed by
 * index (md_bonded_reindex) is read in the atoms' own order.  A bond with
 * r >= R0 contributes nothing and raises MD_F_BOND_BROKEN.  energy/virial
 * ([R], optional) receive the bond energy and virial per replica, reduced in
 * a fixed order.  Each atom sums its own bonds: deterministic, no atomics. */
int md_fene_forces(const md_batch *b, const md_atoms *atoms, const md_bonds *bonds,
                   double K, double R0, double *energy, double *virial, void *ws,
                   size_t ws_bytes, uint32_t *status, void *stream);

/* Cosine angle term of the ring-polymer melt (Sec. 4 of the paper: a cosine
 * potential on the triples of consecutive beads): for a triple (a, b, c) with
 * d1 = x_a - x_b, d2 = x_c - x_b (minimum image) and cos t = d1.d2/(|d1||d2|),
 * U = K (1 + cos t), zero for a straight triple, and the forces are -grad U.
 * Forces are ADDED to fx, fy, fz.  A table keyed by id needs atoms->where,
 * and the ids of replica r must then be the range [atom_off[r],
 * atom_off[r+1]) (that work is spread over ids); a table keyed by index
 * (md_bonded_reindex) is read in the atoms' own order.  A triple with a
 * zero-length bond vector contributes nothing and raises MD_F_NONFINITE.
 * energy/virial ([R], optional) receive the angle energy and virial
 * (d1.F_a + d2.F_c per triple, zero up to rounding: the term is scale
 * invariant) per replica, reduced in a fixed order.  Each atom sums its own
 * share of its triples: deterministic, no atomics.  MD_EINVAL for a missing
 * pointer, max_angles outside 1 .. MD_MAX_ANGLES, an unknown order or K
 * negative or not finite. */
int md_angle_forces(const md_batch *b, const md_atoms *atoms, const md_angles *angles,
                    double K, double *energy, double *virial, void *ws, size_t ws_bytes,
                    uint32_t *status, void *stream);

/* md_fene_forces and md_angle_forces in one pass over the atoms, for tables
 * keyed by index (md_bonded_reindex; MD_EINVAL otherwise): each atom sums its
 * bonds (K, R0) and its angle triples (Ka) and updates its force once.  The
 * results equal the two calls in sequence bit for bit (forces, flags, and
 * the energy/virial outputs of each term, all optional). */
int md_bonded_forces(const md_batch *b, const md_atoms *atoms, const md_bonds *bonds,
                     double K, double R0, const md_angles *angles, double Ka,
                     double *energy_bond, double *virial_bond, double *energy_angle,
                     double *virial_angle, void *ws, size_t ws_bytes, uint32_t *status,
                     void *stream);

/* Bonded tables in the atoms' current (cell-sorted) order: for every atom
 * at index i of a replica whose gate is set (every replica when gate is
 * NULL; pass md_cell_sort's gate), copies the MD_BY_ID tables' column id[i]
 * into column i of the outputs, with every member id translated to its
 * current index through atoms->where.  Unused slots are set to -1.  The
 * outputs then form MD_BY_INDEX tables of the same max_bonds / max_angles for
 * md_fene_forces and md_angle_forces, which read them coalesced and gather
 * positions from nearby cells.  Call after each md_cell_sort that moved
 * atoms.  bonds or angles may be NULL (their outputs are then not touched);
 * outputs: bond_count [N], bond_partner [max_bonds N], angle_count [N],
 * angle_tri [3 max_angles N].  Member ids must lie in [0, N).  MD_EINVAL for
 * an input table not keyed by id, a missing output or atoms->id/where, or a
 * slot count out of range. */
int md_bonded_reindex(const md_batch *b, const md_atoms *atoms, const md_bonds *bonds,
                      int32_t *bond_count, int32_t *bond_partner, const md_angles *angles,
                      int32_t *angle_count, int32_t *angle_tri, const uint32_t *gate,
                      void *stream);

/* Langevin thermostat in force form (Sec. 4: particles equilibrated to a
 * target temperature T): F_i += -gamma m_i v_i + sqrt(2 gamma m_i T / dt) xi_i
 * with v the velocity at the time of the force evaluation.  xi_i are three
 * standard normals from the counter-based generator Philox4x32-10 (Salmon,
 * Moraes, Dror, Shaw, SC 2011) with key (seed low, seed high) and counters
 * (id_i, step low, step high, 0) and (..., 1); each pair of 32-bit outputs
 * forms a 53-bit uniform (w0 w1 >> 11 + 1/2) 2^-53 in (0, 1), and Box-Muller
 * maps two uniforms to two normals (the fourth normal is unused).  `step`
 * (device, one uint64) is read by every atom and then advanced by one, so
 * calls replayed from a captured graph draw fresh noise.  mass: [ntypes]. */
int md_langevin(const md_batch *b, const md_atoms *atoms, const double *mass,
                int32_t ntypes, double gamma, double temperature, double dt,
                uint64_t seed, uint64_t *step, uint32_t *status, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* MD_H */
