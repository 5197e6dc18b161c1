// program.cpp -- validation and canonicalisation of postfix programs.
#include "program.hpp"

#include <cstdio>

namespace salt {

static salt_status fail(std::string *err, salt_status s, const char *fmt, int a = 0, int b = 0) {
    if (err) {
        char buf[160];
        std::snprintf(buf, sizeof buf, fmt, a, b);
        *err = buf;
    }
    return s;
}

salt_status compile_program(const uint32_t *prog, int32_t len, int32_t n_operands,
                            int32_t n_scalars, Program *out, std::string *err) {
    if (!prog) return fail(err, SALT_ERR_ARG, "program pointer is NULL");
    if (len < 1 || len > SALT_MAX_TOKENS)
        return fail(err, SALT_ERR_PROGRAM, "program length %d outside 1..%d", len, SALT_MAX_TOKENS);
    if (n_operands < 0 || n_operands > SALT_MAX_OPERANDS)
        return fail(err, SALT_ERR_ARG, "n_operands %d outside 0..%d", n_operands, SALT_MAX_OPERANDS);
    if (n_scalars < 0 || n_scalars > SALT_MAX_SCALARS)
        return fail(err, SALT_ERR_ARG, "n_scalars %d outside 0..%d", n_scalars, SALT_MAX_SCALARS);

    Program p;
    int op_canon[SALT_MAX_OPERANDS], sc_canon[SALT_MAX_SCALARS];
    for (int k = 0; k < SALT_MAX_OPERANDS; ++k) op_canon[k] = -1, p.op_map[k] = 0;
    for (int j = 0; j < SALT_MAX_SCALARS; ++j) sc_canon[j] = -1, p.sc_map[j] = 0;

    int depth = 0;
    for (int t = 0; t < len; ++t) {
        const uint32_t op = prog[t] & 0xffu, arg = prog[t] >> 8;
        p.sarg[t] = 0;
        p.sarg_raw[t] = 0;
        if (op == SALT_OP_LOAD) {
            if (arg >= (uint32_t)n_operands)
                return fail(err, SALT_ERR_PROGRAM, "token %d loads operand %d, out of range", t, (int)arg);
            if (depth >= SALT_MAX_STACK)
                return fail(err, SALT_ERR_PROGRAM, "token %d exceeds the stack limit %d", t, SALT_MAX_STACK);
            if (op_canon[arg] < 0) {
                op_canon[arg] = p.n_loads;
                p.op_map[p.n_loads++] = (int32_t)arg;
            }
            p.canon[t] = SALT_TOKEN(SALT_OP_LOAD, op_canon[arg]);
            p.code[t] = (uint8_t)(op_canon[arg] * 8 + depth);
            p.code_raw[t] = (uint8_t)(arg * 8 + depth);
            p.load_mask |= 1u << arg;
            ++depth;
        } else if (op == SALT_OP_SCALAR) {
            if (arg >= (uint32_t)n_scalars)
                return fail(err, SALT_ERR_PROGRAM, "token %d reads scalar %d, out of range", t, (int)arg);
            if (depth >= SALT_MAX_STACK)
                return fail(err, SALT_ERR_PROGRAM, "token %d exceeds the stack limit %d", t, SALT_MAX_STACK);
            if (sc_canon[arg] < 0) {
                sc_canon[arg] = p.n_scal;
                p.sc_map[p.n_scal++] = (int32_t)arg;
            }
            p.canon[t] = SALT_TOKEN(SALT_OP_SCALAR, sc_canon[arg]);
            p.code[t] = (uint8_t)(kCodeScalar + depth);
            p.code_raw[t] = p.code[t];
            p.sarg[t] = (uint8_t)sc_canon[arg];
            p.sarg_raw[t] = (uint8_t)arg;
            ++depth;
        } else if (op == SALT_OP_ADD || op == SALT_OP_SUB || op == SALT_OP_MUL) {
            if (arg != 0)
                return fail(err, SALT_ERR_PROGRAM, "token %d: binary operation with argument %d", t, (int)arg);
            if (depth < 2)
                return fail(err, SALT_ERR_PROGRAM, "token %d: stack underflow (depth %d)", t, depth);
            p.canon[t] = SALT_TOKEN(op, 0);
            p.code[t] = (uint8_t)(kCodeBinary + 8 * (int)(op - SALT_OP_ADD) + (depth - 2));
            p.code_raw[t] = p.code[t];
            --depth;
        } else {
            return fail(err, SALT_ERR_PROGRAM, "token %d has unknown opcode %d", t, (int)op);
        }
        if (depth > p.stack_need) p.stack_need = depth;
    }
    if (depth != 1)
        return fail(err, SALT_ERR_PROGRAM, "program leaves %d values on the stack, not 1", depth);
    p.len = len;
    *out = p;
    return SALT_OK;
}

}  // namespace salt
