// ctx.h -- the single-lattice context behind the opaque hlb_ctx handle
// (shared by the solver and the surrogate entry points).
#pragma once

#include "kernels.h"

struct hlb_ctx {
    hlb::Device D;
    hlb::PhysParams p;
    bool have_params;
    bool have_fields;
    int status;
    char msg[512];
    size_t state_bytes;
    void *ws;         // the caller's workspace and its size
    size_t ws_bytes;
    // bumped by every call that changes the state or the parameters from
    // outside the surrogate driver (which keeps a Q history per context)
    unsigned long long version;
};
