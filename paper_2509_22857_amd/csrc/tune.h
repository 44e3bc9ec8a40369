// Tunable launch choices (process-wide), set through ckc_tune_set by the
// autotuner; every choice gives bit-identical results.
#pragma once

enum TuneKnob {
    TK_CONV_OUTS = 0,  // outputs per wave of the convolution contraction: 8 or 16
    TK_CONV_IMGS,      // most images per contraction workgroup: 1, 2 or 4
    TK_KS_BATCH,       // rotated inputs per key-switching launch in a convolution: 8 .. 64
    TK_CONV_FUSE,      // 1: one contraction launch covers every output group of a 3x3 layer
    TK_CONV_ROWS,      // polynomials per contraction wave: 1, or 2 (one codebook read per two products)
    TK_COUNT
};

int tune_value(TuneKnob k);
