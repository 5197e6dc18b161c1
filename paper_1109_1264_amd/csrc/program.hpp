// program.hpp -- host-side compilation of a postfix expression program.
//
// The paper builds the expression tree at compile time and an execute
// function picks a loop template for it (Sec. 4.1, Fig. 2; the choice by
// register use, Sec. 4.3). Here the tree arrives at run time as postfix
// tokens; this module validates it, renumbers operands and scalars in order
// of first use (so equal tree shapes share one compiled kernel), and encodes
// it for the generic interpreter kernel. Host only: no HIP calls.
#pragma once

#include <cstdint>
#include <string>

#include "salt.h"

namespace salt {

// Interpreter instruction codes: each names the operation together with the
// stack slot it writes, so the kernel's register file is indexed by constants.
//   LOAD k into slot s   -> k*8 + s          (0..63)
//   SCALAR into slot s   -> 64 + s           (64..71); value index in sarg[]
//   ADD/SUB/MUL          -> 72 + 8*op + s    (op 0..2, s = slot of the left
//                           operand; the right operand is in slot s + 1)
constexpr int kCodeScalar = 64;
constexpr int kCodeBinary = 72;
constexpr int kNumCodes = 96;

struct Program {
    int32_t len = 0;
    uint32_t canon[SALT_MAX_TOKENS];  // tokens with canonical operand/scalar numbers
    int32_t n_loads = 0;              // distinct operands read
    int32_t n_scal = 0;               // distinct scalars read
    int32_t op_map[SALT_MAX_OPERANDS];  // canonical operand -> caller's index
    int32_t sc_map[SALT_MAX_SCALARS];   // canonical scalar  -> caller's index
    int32_t stack_need = 0;
    uint8_t code[SALT_MAX_TOKENS];    // interpreter codes
    uint8_t sarg[SALT_MAX_TOKENS];    // canonical scalar index for scalar codes
    // The same codes with the caller's operand and scalar numbers (used when
    // several programs share one operand list), and the operands read.
    uint8_t code_raw[SALT_MAX_TOKENS];
    uint8_t sarg_raw[SALT_MAX_TOKENS];
    uint32_t load_mask = 0;           // bit k: caller operand k is read
};

// Validate `prog` against the operand and scalar counts and compile it.
// Returns SALT_OK or SALT_ERR_PROGRAM / SALT_ERR_ARG with a message in *err.
salt_status compile_program(const uint32_t *prog, int32_t len, int32_t n_operands,
                            int32_t n_scalars, Program *out, std::string *err);

}  // namespace salt
