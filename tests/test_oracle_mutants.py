"""The oracle's pins must be able to fail: each case below plants one
plausible mistake in a copy of an oracle module (a dropped term, a wrong sign,
index or norm, a transposed operand, a missing rounding or correction step),
puts the copy's functions in place of the module's for the duration of the
test, and runs the pins of tests/test_oracle.py that cover that module.  At
least one pin has to fail for every mistake.  All on the CPU; the mistakes are
planted in the oracle only."""
import importlib
import inspect
import types

import pytest

from tests import test_oracle as T

PRODUCT_PINS = [
    (T.test_product_dense_bruteforce, ()),
    (T.test_product_closed_forms, ()),
    (T.test_product_indicator_and_ones, ()),
    (T.test_product_integer_exact_and_invariants, ()),
    (T.test_proposition_reuse_equals_plain, ()),
    (T.test_difference_form_rule, ()),
]
LEFT_PINS = [
    (T.test_left_product_dense_and_closed_forms, ()),
    (T.test_left_product_through_the_difference_form, ()),
]
PAGERANK_PINS = [(T.test_pagerank_dense_solve, (s,)) for s in (0, 1, 2)] + [
    (T.test_pagerank_closed_forms, ()),
    (T.test_pagerank_degenerate, ()),
    (T.test_pagerank_mass_conserved, ()),
]
DECODE_PINS = [
    (T.test_codes_golden, ()),
    (T.test_nu_inverse, ()),
    (T.test_tiny_stream_golden, ()),
    (T.test_roundtrip_web, ()),
    (T.test_roundtrip_crafted, ()),
    (T.test_roundtrip_long_row, ()),
    (T.test_corrupt_streams, ()),
] + [(T.test_roundtrip_params, p) for p in ((7, 3, 4, 3), (1, 1, 2, 1), (0, 0, 3, 2), (15, 15, 8, 5))]
MLP_PINS = [
    (T.test_bf16_rounding_values, ()),
    (T.test_gelu_identities, ()),
    (T.test_mlp_gradient_finite_differences, ()),
    (T.test_mlp_quantized_close_to_exact, ()),
    (T.test_adam_first_step_closed_form, ()),
    (T.test_mlp_inputs_enter_as_bf16, ()),
    (T.test_mlp_weights_enter_as_bf16, ()),
    (T.test_mlp_hidden_layer_enters_as_bf16, ()),
    (T.test_mlp_backward_operands_are_bf16, ()),
]
FEATURE_PINS = [
    (T.test_row_stats_match_lists, ()),
    (T.test_structural_closed_forms_star, ()),
    (T.test_structural_depth_input_is_normalised, ()),
    (T.test_trajectory_and_target_single_mode, ()),
    (T.test_restart_vector_perfect_and_floor, ()),
]
RESTART_PINS = [
    (T.test_restarted_zero_and_rejected_predictions_follow_plain_method, ()),
    (T.test_restarted_perfect_prediction_converges_after_restart, ()),
    (T.test_restarted_matches_dense_fixed_point, ()),
    (T.test_restart_kept_only_under_the_contraction_bound, ()),
]

BICLIQUE_PINS = [
    (T.test_biclique_closed_form_complete_bipartite, ()),
    (T.test_biclique_dense_bruteforce_and_lists, ()),
    (T.test_biclique_indicator_and_ones, ()),
    (T.test_biclique_miner_partitions_the_edges, ()),
]

# (id, oracle module, source text, mistaken text, pins)
MUTANTS = [
    # left product: x A by definition, and through c = x (I - R)^{-1}
    ("left-product-not-transposed", "oracle.product",
     "return np.bincount(np.asarray(col, dtype=np.int64), weights=x[rows], minlength=n).astype(np.float64)",
     "return np.bincount(rows, weights=x[np.asarray(col, dtype=np.int64)], minlength=n).astype(np.float64)",
     LEFT_PINS),
    ("left-recurrence-forward-order", "oracle.product", "    for i in range(n - 1, -1, -1):\n        if r[i] >= 0:",
     "    for i in range(n):\n        if r[i] >= 0:", LEFT_PINS),
    ("left-recurrence-dropped", "oracle.product", "            c[r[i]] += c[i]", "            pass", LEFT_PINS),
    ("left-minus-sign", "oracle.product", "            y[j] -= c[i]", "            y[j] += c[i]", LEFT_PINS),
    # biclique format: c_r over C_r, added to the rows of S_r, plus residual edges
    ("biclique-sum-over-S", "oracle.biclique", "C = b.cidx[int(b.cptr[r]):int(b.cptr[r + 1])].astype(np.int64)\n        c[r]",
     "C = b.sidx[int(b.sptr[r]):int(b.sptr[r + 1])].astype(np.int64)\n        c[r]", BICLIQUE_PINS),
    ("biclique-scatter-transposed", "oracle.biclique", "        y[S] += c[r]",
     "        y[b.cidx[int(b.cptr[r]):int(b.cptr[r + 1])].astype(np.int64)] += c[r]", BICLIQUE_PINS),
    ("biclique-residual-dropped", "oracle.biclique", "            y[i] += np.sum(x[R])", "            pass",
     BICLIQUE_PINS),
    ("biclique-lists-residual-dropped", "oracle.biclique",
     "        rows[i].extend(b.rcol[int(b.rptr[i]):int(b.rptr[i + 1])].tolist())", "        pass", BICLIQUE_PINS),
    ("biclique-scatter-set-not-added", "oracle.biclique", "        y[S] += c[r]", "        y[S] = c[r]",
     BICLIQUE_PINS),
    # product: the definition y_i = sum of x over row i, and the reuse algorithm
    ("row-last-entry-dropped", "oracle.product", "y[i] = math.fsum(x[col[a:b]].tolist())",
     "y[i] = math.fsum(x[col[a:b - 1]].tolist())", PRODUCT_PINS),
    ("transposed-operand", "oracle.product",
     "        if b > a:\n            y[i] = math.fsum(x[col[a:b]].tolist())",
     "        for j in col[a:b]:\n            y[int(j)] += x[i]", PRODUCT_PINS),
    ("gather-index-shifted", "oracle.product", "vals = x[np.asarray(col, dtype=np.int64)]",
     "vals = x[(np.asarray(col, dtype=np.int64) + 1) % n]", PRODUCT_PINS),
    ("correction-sign", "oracle.product",
     "y[i] = base + math.fsum(x[plus[i]].tolist()) - math.fsum(x[minus[i]].tolist())",
     "y[i] = base + math.fsum(x[plus[i]].tolist()) + math.fsum(x[minus[i]].tolist())", PRODUCT_PINS),
    ("reference-row-index", "oracle.product", "base = y[r[i]] if r[i] >= 0 else 0.0",
     "base = y[max(r[i] - 1, 0)] if r[i] >= 0 else 0.0", PRODUCT_PINS),
    ("plus-minus-swapped", "oracle.product", "add, sub = sorted(vi - vr), sorted(vr - vi)",
     "add, sub = sorted(vr - vi), sorted(vi - vr)", PRODUCT_PINS),
    ("fallback-rule-dropped", "oracle.product", "if len(add) + len(sub) < len(vi):", "if True:",
     PRODUCT_PINS),
    # PageRank, Eq. (1) with dangling mass sent to the teleport vector
    ("dangling-mass-dropped", "oracle.pagerank", "beta * (y + delta * v)", "beta * y", PAGERANK_PINS),
    ("beta-swapped", "oracle.pagerank", "p_new = (1.0 - beta) * v + beta * (y + delta * v)",
     "p_new = beta * v + (1.0 - beta) * (y + delta * v)", PAGERANK_PINS),
    ("degrees-transposed", "oracle.pagerank",
     "return np.bincount(np.asarray(col, dtype=np.int64), minlength=n).astype(np.int64)",
     "return np.diff(np.asarray(rowptr, dtype=np.int64))", PAGERANK_PINS),
    ("residual-max-norm", "oracle.pagerank", "resid = float(np.sum(np.abs(p_new - p)))",
     "resid = float(np.max(np.abs(p_new - p)))", PAGERANK_PINS),
    ("teleport-ignored", "oracle.pagerank",
     "v = np.full(n, 1.0 / n) if teleport is None else np.asarray(teleport, dtype=np.float64)\n    p = v.copy()",
     "v = np.full(n, 1.0 / n)\n    p = v.copy()", PAGERANK_PINS),
    ("stale-dangling-mass", "oracle.pagerank", "delta = float(np.sum(p[dangling]))",
     "delta = float(np.sum(v[dangling]))", PAGERANK_PINS),
    # the decoder's codes
    ("gamma-offset", "oracle.bvdecode", "return ((1 << b) | self.read_bits(b)) - 1",
     "return (1 << b) | self.read_bits(b)", DECODE_PINS),
    ("zeta-threshold", "oracle.bvdecode", "if z >= thr:", "if z > thr:", DECODE_PINS),
    ("zeta-bucket-base", "oracle.bvdecode", "left = 1 << (h * k)", "left = 1 << (h * k + 1)", DECODE_PINS),
    ("nu-parity-swapped", "oracle.bvdecode", "return u // 2 if u % 2 == 0 else -((u + 1) // 2)",
     "return u // 2 if u % 2 == 1 else -((u + 1) // 2)", DECODE_PINS),
    ("bits-not-shifted", "oracle.bvdecode", "v = (v << 1) | int(b)", "v = v | int(b)", DECODE_PINS),
    ("copy-blocks-parity", "oracle.bvdecode", "            if keep:                      # b even: the rest is copied\n",
     "            if not keep:\n", DECODE_PINS),
    ("copy-block-length-offset", "oracle.bvdecode", "ln = br.gamma() if b == 0 else br.gamma() + 1",
     "ln = br.gamma() + 1", DECODE_PINS),
    ("interval-gap", "oracle.bvdecode", "s = prev_last + 2 + br.gamma()", "s = prev_last + 1 + br.gamma()",
     DECODE_PINS),
    ("interval-length-offset", "oracle.bvdecode", "ln = br.gamma() + Lmin", "ln = br.gamma() + Lmin - 1",
     DECODE_PINS),
    ("residual-gap", "oracle.bvdecode", "j = prev + 1 + br.zeta(zk)", "j = prev + br.zeta(zk)", DECODE_PINS),
    ("first-residual-not-relative", "oracle.bvdecode", "j = i + nu_inv(br.zeta(zk))", "j = nu_inv(br.zeta(zk))",
     DECODE_PINS),
    ("skipped-stat", "oracle.bvdecode", "stats[i, 1] = len(ref) - len(copied)", "stats[i, 1] = len(copied)",
     FEATURE_PINS),
    ("depth-stat", "oracle.bvdecode", "stats[i, 0] = depth[i]", "stats[i, 0] = g", FEATURE_PINS),
    # the sampled-row product used at full size
    ("sampled-rows-last-entry-dropped", "oracle.product",
     "out[k] = math.fsum(x[col[a:b]].tolist()) if b > a else 0.0",
     "out[k] = math.fsum(x[col[a:b - 1]].tolist()) if b > a else 0.0", PRODUCT_PINS),
    # the network
    ("bf16-truncates", "oracle.mlp", "u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000",
     "u = u & 0xFFFF0000", MLP_PINS),
    ("gelu-sign", "oracle.mlp", "return z * _sigma(GELU_A * z)", "return z * _sigma(-GELU_A * z)", MLP_PINS),
    ("gelu-grad-term-dropped", "oracle.mlp", "return s + GELU_A * z * s * (1.0 - s)", "return s", MLP_PINS),
    ("adam-bias-correction-dropped", "oracle.mlp", "mh = self.m / (1 - self.b1 ** self.t)", "mh = self.m",
     MLP_PINS),
    ("backprop-weight-transposed", "oracle.mlp", "dh1 = dz2q @ p[\"W2\"]", "dh1 = dz2q @ p[\"W2\"].T",
     MLP_PINS),
    ("bias-grad-from-wrong-layer", "oracle.mlp", "g[\"b1\"] = dz1.sum(axis=0)", "g[\"b1\"] = dh1.sum(axis=0)",
     MLP_PINS),
    ("x-not-rounded", "oracle.mlp", "xq = q(X)", "xq = X", MLP_PINS),
    ("h1-not-rounded", "oracle.mlp", "h1q = q(h1)", "h1q = h1", MLP_PINS),
    ("dz2-not-rounded", "oracle.mlp", "dz2q = q(dz2)", "dz2q = dz2", MLP_PINS),
    ("dz1-not-rounded", "oracle.mlp", "dz1q = q(dz1)", "dz1q = dz1", MLP_PINS),
    ("w3-not-rounded", "oracle.mlp", 'WEIGHTS = ("W1", "W2", "w3")', 'WEIGHTS = ("W1", "W2")', MLP_PINS),
    ("b2-grad-from-rounded-delta", "oracle.mlp", 'g["b2"] = dz2.sum(axis=0)', 'g["b2"] = dz2q.sum(axis=0)',
     MLP_PINS),
    # the network's inputs, target and restart vector
    ("trajectory-norm", "oracle.features", "delta = float(np.sum(np.abs(pK - pK1)))",
     "delta = float(np.sqrt(np.sum((pK - pK1) ** 2)))", FEATURE_PINS),
    ("target-sign", "oracle.features", "return pK.size * (p_star - pK) / delta",
     "return pK.size * (pK - p_star) / delta", FEATURE_PINS),
    ("restart-not-normalised", "oracle.features", "return q / np.sum(q)", "return q", FEATURE_PINS),
    ("restart-step-unscaled", "oracle.features", "q = np.maximum(pK + s * delta / pK.size, FLOOR * pK)",
     "q = np.maximum(pK + s * delta, FLOOR * pK)", FEATURE_PINS),
    ("neighbour-mean-of-indegree", "oracle.features",
     "F[:, 6] = np.log1p(_product.matvec(rowptr, col, d) / den)",
     "F[:, 6] = np.log1p(_product.matvec(rowptr, col, indeg) / den)", FEATURE_PINS),
    ("depth-input-scale", "oracle.features", "F[:, 2] = stats[:, 0] / float(max(R, 1))",
     "F[:, 2] = stats[:, 0] / float(max(R, 1) + 1)", FEATURE_PINS),
    ("trajectory-lag", "oracle.features", "T[:, 2] = n * (pK1 - pK2) / delta", "T[:, 2] = n * (pK - pK2) / delta",
     FEATURE_PINS),
    ("log-input-unscaled", "oracle.features", "T[:, 0] = np.log(n * pK)", "T[:, 0] = np.log(pK)", FEATURE_PINS),
    ("skipped-count-reversed", "oracle.features", "out[v, 1] = len(Lr - Lv)", "out[v, 1] = len(Lv - Lr)",
     FEATURE_PINS),
    # learned restarts: the probe rule and the product count
    ("probe-rule-inverted", "oracle.restart", "if r < beta * delta:", "if r >= beta * delta:", RESTART_PINS),
    ("probe-rule-loose", "oracle.restart", "if r < beta * delta:", "if r < 2.0 * delta:", RESTART_PINS),
    ("probe-rule-without-beta", "oracle.restart", "if r < beta * delta:", "if r < delta:", RESTART_PINS),
    ("rejected-probe-not-counted", "oracle.restart", "products=t + rejected", "products=t", RESTART_PINS),
    ("restart-without-probe-step", "oracle.restart", "            p, resid = q, r\n            t += 1\n",
     "            p, resid = p_new, r\n            t += 1\n", RESTART_PINS),
]


def _mutant(modname, old, new):
    mod = importlib.import_module(modname)
    src = inspect.getsource(mod)
    assert src.count(old) == 1, "the text to mutate must occur once in %s: %r" % (modname, old)
    m = types.ModuleType(modname + "_mutant")
    m.__package__ = mod.__package__
    m.__file__ = mod.__file__
    exec(compile(src.replace(old, new), mod.__file__ + " (mutant)", "exec"), m.__dict__)
    return mod, m


@pytest.mark.parametrize("name,modname,old,new,pins", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_fails_a_pin(name, modname, old, new, pins, monkeypatch):
    mod, m = _mutant(modname, old, new)
    for attr, obj in vars(m).items():
        if (inspect.isfunction(obj) or inspect.isclass(obj)) and getattr(obj, "__module__", "") == m.__name__:
            monkeypatch.setattr(mod, attr, obj)
    failed = []
    for pin, args in pins:
        try:
            pin(*args)
        except Exception as e:  # an assertion, or the mistake breaking the computation outright
            failed.append((pin.__name__, type(e).__name__))
            break
    assert failed, "no pin fails when the oracle has the mistake %r" % name


def test_unmutated_oracle_passes_every_pin():
    for pin, args in PRODUCT_PINS + PAGERANK_PINS + DECODE_PINS + MLP_PINS + FEATURE_PINS + RESTART_PINS:
        pin(*args)
