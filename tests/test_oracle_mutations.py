"""Mutation check of the oracle's pins (CPU only).

Each case plants one plausible mistake in a private copy of
oracle/hth_oracle.c (a dropped term, a wrong index, a transposed operand, a
wrong sign), builds it into its own library, and runs the pins named for it
against that library: each of them must fail.  The unmodified oracle passes
every pin (tests/test_oracle_pins.py), so a pin that fails here is one that
tells the planted mistake apart from the paper's definition.
"""
import importlib.util
import os
import subprocess

import pytest

import test_oracle_pins as pins

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_DIR = os.path.join(ROOT, "oracle")
SRC = os.path.join(ORACLE_DIR, "hth_oracle.c")
WIDTHS = pins.WIDTHS

# name -> (text in hth_oracle.c, replacement, pins that must catch it)
# A pin is (function, list of keyword-argument sets); it catches the mutant
# when one of its calls raises AssertionError.
_W = [dict(width=w) for w in WIDTHS]
_WB = [dict(width=w, b=b) for w in WIDTHS for b in (8, 4)]

MUTANTS = {
    # NH (§3.2): a carry from the low half into the high half
    "nh_carry": (
        "uint64_t hi = (((x >> W) & hm) + ((s >> W) & hm)) & hm;",
        "uint64_t hi = ((((x & word_mask(W)) + (s & word_mask(W))) >> W) & hm);",
        [(pins.test_nh_closed_forms, [{}])]),
    # Combine (§5.1): one entry of the printed T
    "t_entry": (
        "{{1, 0, 1, 1, 2, 1, 4},",
        "{{1, 0, 1, 1, 2, 1, 5},",
        [(pins.test_combine_matrix_p, [dict(width=16)])]),
    # Combine: the sign of the sum
    "combine_sign": (
        "for (unsigned c = 0; c < sh->e; c++) acc += (uint64_t)sh->T[t][c] * h[c];",
        "for (unsigned c = 0; c < sh->e; c++) acc -= (uint64_t)sh->T[t][c] * h[c];",
        [(pins.test_zero_entropy_closed_forms, _W)]),
    # Encode (§3.3): a parity entry that breaks the distance of the HH24 code
    "p_entry": (
        "{{1, 4, 1, 2, 1, 5, 1},\n      {1, 5, 4, 5, 2, 4, 5}},",
        "{{1, 4, 1, 2, 1, 5, 1},\n      {1, 5, 4, 5, 2, 5, 5}},",
        [(pins.test_code_distance_binary_image, [dict(width=24)])]),
    # Encode: the binary image transposed
    "image_transposed": (
        "if (mbit(sh->P[r][c], u, v)) sum += X[c * w + v];",
        "if (mbit(sh->P[r][c], v, u)) sum += X[c * w + v];",
        [(pins.test_zero_entropy_closed_forms, _W)]),
    # Lane map (§2): instance j read as the j-th run of d*w words
    "lane_map": (
        "X[c * w + u] = words[g * xw + (uint64_t)(c * w + u) * b + j];",
        "X[c * w + u] = words[g * xw + (uint64_t)j * (d * w) + c * w + u];",
        [(pins.test_zero_entropy_closed_forms, _W)]),
    # Hash (§3.3 step 2): a key picked by the sub-word alone, shared by items
    "ehc_key_by_subword": (
        "nh_counted(W, Y[c * w + u], S_ehc[c * w + u], MUL_EHC)",
        "nh_counted(W, Y[c * w + u], S_ehc[u], MUL_EHC)",
        [(pins.test_ehc_swap_pair_w8, [{}]), (pins.test_ehc_single_key_closed_form, _WB)]),
    # Hash: one key per item instead of one per word
    "ehc_key_by_item": (
        "nh_counted(W, Y[c * w + u], S_ehc[c * w + u], MUL_EHC)",
        "nh_counted(W, Y[c * w + u], S_ehc[c * w], MUL_EHC)",
        [(pins.test_ehc_single_key_closed_form, _WB)]),
    # Tree (§5.2): keys not indexed by level
    "tree_key_level": (
        "node += nh_counted(st->W, st->items[level * f1 + i], st->S_tree[level * f1 + i], MUL_TREE);",
        "node += nh_counted(st->W, st->items[level * f1 + i], st->S_tree[i], MUL_TREE);",
        [(pins.test_eq1_binary_tree_power_of_two, [{}])]),
    # Tree: the last child hashed like the others
    "last_child_hashed": (
        "uint64_t node = v; /* the f-th child is added without a product */",
        "uint64_t node = nh(st->W, v, st->S_tree[level * f1]);",
        [(pins.test_eq1_binary_tree_power_of_two, [{}])]),
    # Final NH (§5.2, §6.1): keys shared by the instances
    "final_key_no_instance": (
        "uint64_t key = S_final[(((uint64_t)t * L + l) * f1 + i) * b + j];",
        "uint64_t key = S_final[(((uint64_t)t * L + l) * f1 + i) * b];",
        [(pins.test_instance_swap_no_collisions, _WB), (pins.test_final_single_key_closed_form, _WB)]),
    # Final NH: keys not indexed by level
    "final_key_no_level": (
        "uint64_t key = S_final[(((uint64_t)t * L + l) * f1 + i) * b + j];",
        "uint64_t key = S_final[(((uint64_t)t * L) * f1 + i) * b + j];",
        [(pins.test_final_single_key_closed_form, _WB)]),
    # Final NH: positions and instances transposed
    "final_key_transposed": (
        "uint64_t key = S_final[(((uint64_t)t * L + l) * f1 + i) * b + j];",
        "uint64_t key = S_final[((uint64_t)t * L + l) * f1 * b + j * f1 + i];",
        [(pins.test_final_single_key_closed_form, _WB)]),
    # Tail (§6.1): Toeplitz offset dropped
    "toeplitz_offset": (
        "tl = (tl + nh_counted(W, words[m0 + q], S_tail[t + q], MUL_TAIL)) & m;",
        "tl = (tl + nh_counted(W, words[m0 + q], S_tail[q], MUL_TAIL)) & m;",
        [(pins.test_b4_tail_only_closed_form, _W)]),
    # Length term (§2: the length is appended) dropped
    "length_dropped": (
        "out[t] = (F[t] + tl + ln) & m;",
        "out[t] = (F[t] + tl) & m;",
        [(pins.test_lengths_separate_and_padding, _W)]),
    # Length key shared by the output words
    "length_key_shared": (
        "uint64_t ln = nh_counted(W, len_value, S_len[t], MUL_LEN);",
        "uint64_t ln = nh_counted(W, len_value, S_len[0], MUL_LEN);",
        [(pins.test_b4_tail_only_closed_form, _W)]),
    # Executions counted in words: a partial last word completes an execution
    "exec_in_words": (
        "uint64_t n_exec = len / xb;",
        "uint64_t n_exec = nw / (xb / 8);",
        [(pins.test_zero_entropy_closed_forms, _W)]),
}


def _build(name, tmp_path):
    src = open(SRC).read()
    old, new, _ = MUTANTS[name]
    assert src.count(old) == 1, f"{name}: the text to mutate is not unique in the oracle (or is gone)"
    path = tmp_path / f"{name}.c"
    path.write_text(src.replace(old, new))
    lib = tmp_path / f"lib_{name}.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-I", ORACLE_DIR, "-shared", "-fPIC",
                    "-o", str(lib), str(path), "-lpthread"], check=True)
    spec = importlib.util.spec_from_file_location(f"oracle_mutant_{name}", os.path.join(ORACLE_DIR, "__init__.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    mod.LIB_PATH = str(lib)
    mod._lib = None
    return mod


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_fails_its_pins(name, tmp_path):
    """Every pin named for the mutant fails on it (for at least one of its
    parameter sets)."""
    mod = _build(name, tmp_path)
    missed = []
    for fn, kwargs_list in MUTANTS[name][2]:
        for kw in kwargs_list:
            try:
                fn(oracle_lib=mod, **kw)
            except AssertionError:
                break
        else:
            missed.append(fn.__name__)
    assert not missed, f"mutant {name} passed {missed}"
