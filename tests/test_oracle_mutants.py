"""Planted mistakes in a copy of the oracle must each fail at least one pin.

Each mutant is a one-token edit of oracle.c (a dropped term, a flipped sign or
comparison, a transposed index), compiled on the CPU into a temporary library.
The real oracle.c is never modified.
"""
import os

import pytest

import oracle
from tests import pins

MUTANTS = {
    "sort_ascending": ("if (a->cnt != b->cnt) return a->cnt > b->cnt ? -1 : 1;",
                       "if (a->cnt != b->cnt) return a->cnt < b->cnt ? -1 : 1;"),
    "tie_descending_key": ("return (a->key > b->key) - (a->key < b->key);",
                           "return (a->key < b->key) - (a->key > b->key);"),
    "rank_not_inverse": ("for (int32_t r = 0; r < n_keys; ++r) rank[perm[r]] = r;",
                         "for (int32_t r = 0; r < n_keys; ++r) rank[r] = perm[r];"),
    "recode_identity": ("C_new[j] = (k >= 0 && k < n_keys) ? rank[k] : k;", "C_new[j] = k;"),
    "permute_transposed": ("for (int32_t r = 0; r < n_keys; ++r) out[r] = col[perm[r]];\n}\n\nvoid oracle_permute_i8",
                           "for (int32_t r = 0; r < n_keys; ++r) out[perm[r]] = col[r];\n}\n\nvoid oracle_permute_i8"),
    "filter_le": ("if (!(c < cat_lt)) continue;", "if (!(c <= cat_lt)) continue;"),
    "group_ignored": ("      g = c;\n", "      g = 0;\n"),
    "count_dropped": ("    sum[g] += (int64_t)price[k];\n    count[g] += 1;", "    sum[g] += (int64_t)price[k];"),
    "group_sum_wrong_index": ("sum[g] += (int64_t)V[j];", "sum[g] += (int64_t)V[g];"),
    "invalid_key_joined": ("    if (k < 0 || k >= n_rows) continue;\n    const int32_t c = category[k];",
                           "    if (k < 0) continue;\n    const int32_t c = category[k];"),
    "select_invalid_key": ("    if (k < 0 || k >= n_rows) continue;\n    if (col[k] < lt)", "    if (k < 0) continue;\n    if (col[k] < lt)"),
    "counts_off_by_one": ("    cnt[k] += 1;\n", "    cnt[k] += (k == 0) ? 2 : 1;\n"),
    "materialize_shifted": ("    out[j] = col[k];\n", "    out[j] = col[k > 0 ? k - 1 : k];\n"),
    "materialize_invalid_kept": ("      out[j] = 0;\n      ++invalid;", "      out[j] = k;\n      ++invalid;"),
    "select_le": ("    if (col[k] < lt) out[n++] = j;", "    if (col[k] <= lt) out[n++] = j;"),
    "select_key_not_offset": ("    if (col[k] < lt) out[n++] = j;", "    if (col[k] < lt) out[n++] = k;"),
    "heavy_ascending": ("  qsort(e, (size_t)n_keys, sizeof(freq_entry), by_decreasing_frequency);\n  for (int32_t r = 0; r < k; ++r) {\n    keys[r] = e[r].key;",
                        "  qsort(e, (size_t)n_keys, sizeof(freq_entry), by_decreasing_frequency);\n  for (int32_t r = 0; r < k; ++r) {\n    keys[r] = e[n_keys - 1 - r].key;"),
    "model_no_repeat_term": ("    if (n > 1.0) rep += n - 1.0;", "    if (n > 1.0) rep += n;"),
    "model_cdf_exponent": ("hit += f[i] * (1.0 - pow(1.0 - f[i], (double)lo));", "hit += f[i] * (1.0 - pow(1.0 - f[i], (double)S));"),
    "model_scale_dropped": ("  const double scale = k / (1.0 - f[i]);", "  const double scale = k;"),
    "append_price_shifted": ("    if (price && price_new) price_new[i] = price[i];", "    if (price && price_new) price_new[i] = price[i - 1];"),
    "append_rank_first": ("    rank[i] = i;\n    if (price && price_new)", "    rank[i] = 0;\n    if (price && price_new)"),
    "append_perm_reversed": ("    perm[i] = i;\n    rank[i] = i;", "    perm[i] = n_new - 1 - (i - n_old);\n    rank[i] = i;"),
    "star_filter_inverted": ("    if (!(cust_attr[u] < cust_lt)) continue;", "    if (cust_attr[u] < cust_lt) continue;"),
    "star_customer_as_product": ("    const int32_t g = category[p];\n    if (g < 0 || g >= 16) continue;\n    sum[g] += (int64_t)price[p];",
                                 "    const int32_t g = category[p];\n    if (g < 0 || g >= 16) continue;\n    sum[g] += (int64_t)price[u < n_prod ? u : p];"),
    "heavy_counts_invalid": ("    if (g >= 0 && g < n_keys) e[g].cnt += 1;", "    if (g >= 0 && g < n_keys) e[g].cnt += 1;\n    else if (g == n_keys && n_keys > 0) e[0].cnt += 1;"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(oracle.SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique"
    path = tmp_path / f"mut_{name}.c"
    path.write_text(src.replace(old, new))
    lib = oracle.compile_source(str(path), str(tmp_path / f"libmut_{name}.so"))
    caught = []
    try:
        oracle.use_library(lib)
        for pin in pins.ALL_PINS:
            try:
                pin(oracle)
            except (AssertionError, IndexError, ValueError):
                caught.append(pin.__name__)
    finally:
        oracle.use_library(None)
    assert caught, f"no pin catches mutant {name}"
