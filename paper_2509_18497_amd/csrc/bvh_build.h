// Device buffers of a prepared surfel set and its BVH (owned by gsrad_bvh).
#pragma once

#include <algorithm>

#include "gsrad_internal.h"

namespace gsrad {

struct BvhBuffers {
    SurfRec *rec = nullptr;         // [n] sorted order
    Node *nodes = nullptr;          // [max(n-1,1)]
    float *leafbox = nullptr;       // [n][6] sorted order
    int32_t *leaf_parent = nullptr; // [n]
    int32_t *inv = nullptr;         // [n] original -> sorted
    float *cst = nullptr;           // [n] c = -ln(1-o), original order
    float *opc = nullptr;           // [n] clamped opacity
    float *opraw = nullptr;         // [n] opacity as given
    double *area = nullptr;         // [n] App. E effective area
    float *dado = nullptr;          // [n] d area / d opacity (0 where the clamp is active)
    float *bounds = nullptr;        // [8]
    int *height = nullptr;          // [1] tree height
    void *temp = nullptr;
    size_t temp_bytes = 0;
};

size_t bvh_temp_bytes(int64_t n);
gsrad_status bvh_build(const gsrad_surfels &sf, BvhBuffers &B, hipStream_t st);

}  // namespace gsrad
