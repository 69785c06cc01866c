// Library-internal declarations shared by the host code and the HIP kernels
// of libfskmc (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fskmc {

enum { MODEL_FLIP = 1, MODEL_ZGB = 2 };

// Sweep kernel variants: sites per lane P in {1,4,16}; square blocks
// (8x8, 16x16, 32x32) or 1D rows (64P x 1).
enum Shape { SHAPE_SQ = 0, SHAPE_ROW = 1 };

// Per-block counters, one 16-byte record: accepted events in the block's
// last window (the workload W of Sec. 6), windows that changed the block
// (and were written back), and accepted events since the last reset.
struct BlockCount {
    uint32_t W;
    uint32_t writes;
    unsigned long long events;
};

// Kernel arguments of the single-simulation sweep (one colour, one window).
struct SweepArgs {
    uint8_t* lat;
    const double* table;
    BlockCount* cnt;
    const int32_t* blocks;  // block ids of the active colour
    int n_blocks;
    int Lx, Ly, NBX;
    uint32_t k0, k1, w;
    double dur;
};

// One job of a batched launch; resident in device memory.
struct JobDesc {
    uint8_t* lat;
    const double* table;
    BlockCount* cnt;
    const int32_t* blocks;      // block ids grouped by colour
    const int32_t* colour_off;  // n_colours+1 offsets into blocks
    const int8_t* win_colour;   // per window
    const double* win_dur;      // per window
    uint64_t n_windows;
    uint64_t base_window;       // window index at batch step 0
    int Lx, Ly, NBX;
    uint32_t k0, k1;
    uint32_t item_begin;        // first item of this job in the packed grid
    uint32_t n_items;           // items reserved (max blocks over colours)
    uint32_t pad;
    // persistent batched sweep: colour per block, next window per colour
    // ([n_colours][n_windows+1]), interacting blocks ([nb][8]), epochs
    const int8_t* bcol;
    const int32_t* next_part;
    const int32_t* nbr;
    int32_t* epoch;
    int nb;
    int pad2;
};

// Persistent batched sweep: batch steps [s0, s1) of every job in one launch.
// Items (step, packed item) are taken in step-major order from a 64-bit
// counter, `chunk` at a time; an item of window w waits until every block it
// interacts with has finished its windows before w (per-job epochs).
struct BatchPersistArgs {
    const JobDesc* jobs;
    const uint32_t* item_job;
    uint32_t n_items;           // packed items per step
    uint32_t s0, s1;
    uint32_t chunk;
    unsigned long long* queue;  // zero at launch
    int32_t* abort_flag;
    unsigned long long wait_ticks;
};

// Kernel arguments of the persistent multi-window sweep of one simulation.
struct PersistArgs {
    uint8_t* lat;
    const double* table;
    BlockCount* cnt;
    const int32_t* blocks;      // block ids grouped by colour
    const int32_t* colour_off;  // n_colours+1 offsets into blocks
    const int8_t* win_colour;   // per window
    const double* win_dur;      // per window
    const int32_t* next_part;   // [n_colours][n_windows+1]: first window >= w of colour c
    const int32_t* nbr;         // [n_blocks][8]: blocks that can interact, -1 padded
    int32_t* epoch;             // [n_blocks]: next window each block takes part in
    int32_t* abort_flag;        // raised by a wave whose wait timed out
    int Lx, Ly, NBX;
    uint32_t k0, k1;
    int n_windows;
    int w0, w1;
    int n_waves;                // set by the launcher
    unsigned long long wait_ticks;
};

// Resident persistent sweep (spin flip): every wave keeps the tiles of the
// blocks it owns in LDS for the whole launch; neighbouring blocks exchange only
// their one-site boundary layers through tagged words.
struct ResidentArgs {
    uint8_t* lat;
    const double* table;
    BlockCount* cnt;
    const int8_t* bcol;         // [n_blocks]: colour of each block
    const int8_t* win_colour;   // per window, the array padded to whole dwords
    const double* win_dur;      // per window
    unsigned long long* edge;   // [n_blocks][4]: tag | bits << 32 of the first/last row, first/last column
    const int32_t* owner;       // [n_waves+1] block range of each wave, or null: wave g owns g*bpw .. +bpw-1
    int32_t* abort_flag;        // raised by a wave whose wait timed out
    int Lx, Ly, NBX, NBY, nb;
    uint32_t k0, k1;
    int n_windows;
    int w0, w1;
    int n_waves;                // set by the launcher
    int bpw;                    // blocks per wave, set by the launcher
    unsigned long long wait_ticks;
};

// Nested sweep (Sec. 5, eqs. sublatt2 and opdecomp2): one workgroup per coarse
// cell of the active outer colour; the cell's fine blocks (one wave each per
// inner window) share one LDS tile and run the inner windows [w0, w1) of one
// outer window separated by workgroup barriers.
struct NestedArgs {
    uint8_t* lat;
    const double* table;
    BlockCount* cnt;
    const int8_t* win_colour; // flat colour = outer * k_inner + inner
    const double* win_dur;
    const int32_t* cells;     // coarse cells of the active outer colour, J * NCX + I
    int n_cells;
    int Lx, Ly, NBX, NCX;
    uint32_t k0, k1;
    int w0, w1;
};

// Optional kernel-side timing: when both events are set, the launch records
// them at the kernel's own start and end (hipExtLaunchKernelGGL).
struct LaunchTiming {
    hipEvent_t start = nullptr, stop = nullptr;
};

// Launchers implemented in fskmc_kernels.hip.  They return hipError_t.
hipError_t launch_sweep_single(int model, int P, int shape, int wpg, const SweepArgs& a, hipStream_t s,
                               LaunchTiming tm);
hipError_t launch_sweep_batched(int model, int P, int shape, int wpg, const JobDesc* jobs,
                                const uint32_t* item_job, uint32_t n_items, uint64_t step,
                                hipStream_t s, LaunchTiming tm);
hipError_t launch_sweep_persistent(int model, int P, int shape, int wpg, const PersistArgs& a,
                                   int max_blocks_per_colour, hipStream_t s, LaunchTiming tm);
// hipErrorInvalidConfiguration when the blocks do not fit the resident waves
// (the caller then uses the streaming persistent sweep).
hipError_t launch_sweep_resident(int P, int shape, int wpg, const ResidentArgs& a, hipStream_t s, LaunchTiming tm);
// Waves the resident sweep can keep resident and blocks one wave can hold
// (with an owner array, a.n_waves must be resident_waves(...) and every range
// at most resident_capacity(P) blocks).
int resident_waves(int P, int shape, int wpg);
int resident_capacity(int P);
// Block ranges of the next resident launch from the previous launch's
// workload (one workgroup; see k_rebalance).
hipError_t launch_rebalance(const BlockCount* cnt, unsigned long long* ev_prev, const int8_t* bcol,
                            const int8_t* win_colour, int pw0, int pw1, int first, unsigned long long base,
                            unsigned long long* scan, int32_t* owner, int nb, int use, int n_waves, int cap,
                            hipStream_t s);
// grid == 0: as many workgroups as can be resident on the device.
hipError_t launch_sweep_batched_persistent(int model, int P, int shape, int wpg, const BatchPersistArgs& a,
                                           unsigned grid, hipStream_t s, LaunchTiming tm);
// Lower bound of the resident workgroups of a batched persistent launch
// (sizes the work chunks).
unsigned batched_persistent_grid(int P, int shape, int wpg);
hipError_t launch_epoch_init_batched(const JobDesc* jobs, int n_jobs, hipStream_t s);
// Resident nested sweep (spin flip): every coarse cell is one workgroup for
// the whole launch and keeps its tile in LDS; between outer windows the
// cells exchange their one-site boundary layers through tagged words.
struct NestedResArgs {
    uint8_t* lat;
    const double* table;
    BlockCount* cnt;
    const int8_t* win_colour;   // per window, the array padded to whole dwords
    const double* win_dur;
    const int32_t* ofirst;    // first window of each outer window, n_outer + 1 entries
    unsigned long long* edge; // cells x (cell side / 8) tagged words
    int32_t* abort_flag;
    int Lx, Ly, NBX, NCX, NCY, k_outer;
    uint32_t k0, k1;
    int w0, w1;               // windows of this launch
    int ow0, ow1;             // the outer windows they fall in
    unsigned long long wait_ticks;
};
// hipErrorInvalidConfiguration when the cells do not fit the device at once
// (the caller then launches per outer window).
hipError_t launch_sweep_nested_resident(int P, int c, int k_inner, const NestedResArgs& a, hipStream_t s,
                                        LaunchTiming tm);

// Nested sweep variants: square coarse cells of c x c fine blocks of P*64
// sites with k_inner inner colours; nested_supported() says which exist.
bool nested_supported(int model, int P, int c, int k_inner);
hipError_t launch_sweep_nested(int model, int P, int c, int k_inner, const NestedArgs& a, hipStream_t s,
                               LaunchTiming tm);
hipError_t launch_epoch_init(int32_t* epoch, const int8_t* bcol, const int32_t* next_part, int nb, int n_windows,
                             int w0, hipStream_t s);
hipError_t launch_init(uint8_t* lat, int64_t n, int kind, double p, uint32_t k0, uint32_t k1,
                       hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s);
hipError_t launch_fill_u64(uint64_t* p, int64_t n, uint64_t v, hipStream_t s);
hipError_t launch_observe(const uint8_t* lat, int Lx, int Ly, int dim, const BlockCount* cnt, int n_blocks,
                          unsigned long long* out9, hipStream_t s);

// Static scratch of the allocation-free advance: one file-scope device array
// per GPU, laid out as the FP64 rate table (up to 243 x 14 entries), the
// block ids grouped by colour and one counter record per block.
constexpr int kNoallocMaxBlocks = 65536;
constexpr size_t kNoallocTableBytes = 27648;  // >= 243 * 14 * 8, a multiple of 256
constexpr size_t kNoallocBlocksOff = kNoallocTableBytes;
constexpr size_t kNoallocCountOff = kNoallocBlocksOff + (size_t)kNoallocMaxBlocks * 4;
constexpr size_t kNoallocBytes = kNoallocCountOff + (size_t)kNoallocMaxBlocks * sizeof(BlockCount);
// Device address of the scratch array on `device`, looked up once per device
// (with that device current) and kept; the caller's current device is
// restored afterwards.
hipError_t noalloc_scratch(int device, uint8_t** out);
// n FP64 values written into dst by kernels whose arguments carry them (no
// host-to-device copy).
hipError_t launch_put_f64(double* dst, const double* host, int n, hipStream_t s);
// Block ids grouped by colour for the built-in maps (2 colours (bi+bj)%2, 4
// colours (bi%2)+2(bj%2)), each colour in ascending id order starting at
// off[c].
hipError_t launch_builtin_blocks(int32_t* out, int NBX, int NBY, int n_colours, const int32_t off[4], hipStream_t s);
// W of every block into W (if not null) and the sum of the per-block event
// counters into *events (if not null).
hipError_t launch_noalloc_outputs(const BlockCount* cnt, int nb, uint32_t* W, unsigned long long* events,
                                  hipStream_t s);

}  // namespace fskmc
