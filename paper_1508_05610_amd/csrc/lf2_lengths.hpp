// lf2_lengths.hpp -- line lengths with compiled kernels.
// Every length is 2^a, 3 * 2^a or 5 * 2^a.
#pragma once
#define LF2_LENGTHS(X)                                                                       \
    X(1) X(2) X(3) X(4) X(5) X(6) X(8) X(10) X(12) X(16) X(20) X(24) X(32) X(40) X(48)      \
    X(64) X(80) X(96) X(128) X(160) X(192) X(256) X(320) X(384) X(512) X(640) X(768) X(1024)
// Strided (y / z) passes also take 2048-point lines (2048^3 lattices).
#define LF2_S_LENGTHS(X) LF2_LENGTHS(X) X(2048)
