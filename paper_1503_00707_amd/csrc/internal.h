// internal.h -- host-side structures shared by the library's translation units.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "dvm.h"

namespace dvm {

// Thread-local error text behind dvm_last_error().
int fail(int code, const char *fmt, ...);
void clear_error();

// Morton key of a point on the finest lattice: x bit b -> 3b, y -> 3b+1, z -> 3b+2.
uint64_t morton3(uint64_t x, uint64_t y, uint64_t z);

// Per-cell record read by the step kernels with scalar loads: 128 bytes.
struct alignas(16) DevCell {
    int32_t nbr[6][4];  // neighbour cells per face (-1 padding)
    uint8_t type[6];    // DVM_FACE_*
    uint8_t level;
    uint8_t flags;      // bit 0: the cell has a WALL face
    int32_t pad[6];
};
static_assert(sizeof(DevCell) == 128, "DevCell must stay 128 bytes");

struct Leaf {
    uint64_t key;
    int64_t input;
    int32_t i, j, k;
    uint8_t level;
    uint8_t solid;
};

}  // namespace dvm

struct dvm_mesh {
    int32_t base[3];
    double h0;
    int32_t bc[6];
    int32_t finest;
    int64_t n_leaves;
    std::vector<dvm::Leaf> cells;     // fluid leaves, Morton order
    std::vector<dvm::DevCell> table;  // one record per cell (empty when device_tables)
    double h_min;
    int64_t n_faces[6];
    bool device_tables = false;       // face tables built on the device by each solver (dvm_adapt_tables)
};
