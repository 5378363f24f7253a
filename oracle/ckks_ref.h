/*
 * ckks_ref.h -- the parameter record shared by the oracle's C files.
 *
 * TEST INFRASTRUCTURE ONLY (see ckks_ref.c).
 */
#pragma once
#include <stdint.h>

typedef uint64_t u64;

#define ORC_MAXP 64

typedef struct {
    int32_t logN, N, L, K, dnum, alpha;
    u64 q[ORC_MAXP];      /* combined prime list */
    u64 psi[ORC_MAXP];    /* primitive 2N-th root of unity per prime */
    double scale[ORC_MAXP]; /* scale Delta_l of level l, l = 0..L */
} orc_params;
