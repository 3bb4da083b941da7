"""Regenerate the residual/energy plan: python -m paper_2511_03567_amd.gen

Writes paper_2511_03567_amd/plan.txt, which the library reads at ric_create.
"""
import os
import sys
import time

from . import algebra, compile as comp


def main():
    import argparse
    import pickle
    ap = argparse.ArgumentParser()
    ap.add_argument("--terms-cache", default=None,
                    help="pickle file for the derived spin-free terms (reused when present)")
    args = ap.parse_args()
    t0 = time.time()
    if args.terms_cache and os.path.exists(args.terms_cache):
        with open(args.terms_cache, "rb") as fh:
            e, groups = pickle.load(fh)
    else:
        e, groups = algebra.derive_groups()
        if args.terms_cache:
            with open(args.terms_cache, "wb") as fh:
                pickle.dump((e, groups), fh)
    # the whole residual: both groups merged, doubles merged modulo the pair swap
    r1 = algebra.merge_sf(groups["lin"][0] + groups["quad"][0])
    s2 = algebra.merge_pair_images(algebra.merge_sf(groups["lin"][1] + groups["quad"][1]))
    t1 = time.time()
    plan, res_flops = comp.compile_plan(e, r1, s2, groups=groups)
    text = "\n".join(plan.lines) + "\n"
    here = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    with open(os.path.join(here, "plan.txt"), "w") as fh:
        fh.write(text)
    print(f"terms: E {len(e)}  R1 {len(r1)}  S2 {len(s2)}; derive {t1 - t0:.1f}s; "
          f"plan lines {len(plan.lines)}; residual flops at the cost-model size "
          f"{res_flops:.3e} (ladder {plan.ladder_flops:.3e})", file=sys.stderr)


if __name__ == "__main__":
    main()
