// Tile choices of the autotuner.
//
// A launcher asks for the tile of its kernel family on its workload (radius,
// element type and the volume extents, or the crop list of a batch).  Three
// sources, in order: the candidate the tuner is timing on this thread, the
// choice recorded for that workload, else none (the launcher's heuristic).
//
// Candidates per family (index 0 is always the heuristic):
//   volume families (fused Gaussian, its dot form, grayscale and binary
//   morphology): tz = number of z ranges the volume is split into;
//   batched families (Gaussian, dot, grayscale): tz = slices per work item;
//   separable subgradient (argext, gather): tx x ty column tile and tz
//   slices per work item.
#pragma once

#include <cstdint>
#include <type_traits>

#include "batch.h"

namespace harpia {

enum TuneFamily : int {
    TF_GAUSS = 0,
    TF_GAUSS_DOT,
    TF_GRAY,
    TF_BINARY,
    TF_GAUSS_BATCHED,
    TF_GAUSS_DOT_BATCHED,
    TF_GRAY_BATCHED,
    TF_ARGEXT_BOX,
    TF_GATHER_BOX,
    TF_COUNT
};

struct Tile {
    int32_t tx = 0, ty = 0, tz = 0;
};

const char *tune_family_name(int fam);
int tune_candidates(int fam);
Tile tune_candidate(int fam, int i);

uint64_t tune_key_volume(int fam, int r, int type_code, const int64_t ext[3]);
uint64_t tune_key_batch(int fam, int r, int type_code, const BatchDesc &d);

// The tile for this launch, if the tuner forces one or recorded one.
bool tune_lookup(int fam, uint64_t key, Tile &t);

// Tuner side: force candidate i of `fam` on this thread (i < 0 stops) and
// collect the workload keys the forced launches used; record a tile for all
// of them.
void tune_force(int fam, int i);
void tune_record_seen(int fam, const Tile &t);
void tune_clear();
bool tune_save(const char *path);
bool tune_load(const char *path);
int64_t tune_size();

template <typename T>
constexpr int tune_type_code()
{
    return sizeof(T) == 4 ? 0 : (sizeof(T) == 1 ? 2 : (std::is_same<T, uint16_t>::value ? 1 : (std::is_same<T, _Float16>::value ? 3 : 4)));
}

}  // namespace harpia
