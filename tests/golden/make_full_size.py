"""Writes tests/golden/full_size.json: the CPU oracle's answers on the full-size workloads.

Calls only the oracle (``oracle/``) and the input generators (``synth/``).  Every entry is keyed by the
SHA-256 of the exact input bytes (image, and template where there is one), so a test that regenerates the
inputs can check that they are the ones the answers belong to.

  workload 2  2048x2048 image, one 64x64 template: the plain answer (Eq. 1 at every location); Alg. 2's
              trace and group size; the two-scan search's counts (radius 0 and 2); Alg. 3's conditioning
              for the exact search and as printed (trace, group size, radius, SHA-256 of the conditioned
              image); the exact OptA search's counts (radius = max(blur radius, 2)); the paper's OptA search.
  workload 3  8192x8192 image with clouds, 8 templates of 32, 64 and 128 px: the plain answer of each;
              Alg. 3's conditioning per template size; the exact OptA search's counts per template.
  workload 4  4096x4096 image, 64 templates of sizes 16..128: the plain answer of each.
  workload 5  the first 64 queries of the serving stream (4 resident images, half of the queries cut, half
              noise): the plain answer of each.

Run:  python tests/golden/make_full_size.py [--threads N] [--only 2,3,4,5]
It resumes: entries already in the file are kept.  Several CPU-hours at 8 threads in total.
"""

import argparse
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
from synth import serving_queries, workload  # noqa: E402

OUT = os.path.join(HERE, "full_size.json")
ANSWER = ("y", "x", "rho", "num", "den_t", "den_r")
COUNTS = ("n_locations", "n_centres", "n_eliminated", "n_survivors", "n_computed", "best0")
N_SERVE = 64


def sha(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def pick(d, keys):
    return {k: (float(d[k]) if isinstance(d[k], float) else int(d[k])) for k in keys}


def trace_of(op):
    return [{k: (float(s[k]) if isinstance(s[k], float) else int(s[k])) for k in s} for s in op["trace"]]


def conditioning(img, m, n, paper, threads):
    t0 = time.time()
    op = O.opta(img, m, n, paper=paper, nthreads=threads)
    return op, {"h": op["h"], "w": op["w"], "radius": op["radius"], "cost": int(op["cost"]),
                "trace": trace_of(op), "image_sha256": sha(op["image"]),
                "changed_pixels": int((op["image"] != img).sum()), "seconds": round(time.time() - t0, 1)}


def save(db):
    tmp = OUT + ".tmp"
    with open(tmp, "w") as f:
        json.dump(db, f, indent=1, sort_keys=True)
    os.replace(tmp, OUT)


def log(msg):
    print(time.strftime("%H:%M:%S"), msg, flush=True)


def plain(img, tpl, threads):
    t0 = time.time()
    r = O.full_search(img, tpl, nthreads=threads)
    out = pick(r, ANSWER)
    out["seconds"] = round(time.time() - t0, 1)
    return out


def do_workload2(db, threads):
    w = workload(2)
    img = w["images"][0]
    tpl, loc, _ = w["templates"][0]
    m, n = tpl.shape
    key = "2"
    e = db.setdefault(key, {})
    e["image_sha256"], e["template_sha256"], e["cut"] = sha(img), sha(tpl), list(loc)
    if "plain" not in e:
        e["plain"] = plain(img, tpl, threads)
        save(db)
    if "egs" not in e:
        eg = O.egs(img, m, n, nthreads=threads)
        e["egs"] = {"h": eg["h"], "w": eg["w"], "cost": int(eg["cost"]),
                    "trace": [{k: int(v) if not isinstance(v, bool) else v for k, v in s.items()}
                              for s in eg["trace"]]}
        for radius in (0, 2):
            te = O.te_search(img, tpl, eg["h"], eg["w"], radius=radius, nthreads=threads)
            e["egs"][f"search_radius{radius}"] = pick(te, ANSWER + COUNTS)
        save(db)
    if "opta" not in e:
        op, c = conditioning(img, m, n, False, threads)
        rad = max(op["radius"], 2)
        s = O.opta_search(img, op["image"], tpl, op["h"], op["w"], rad, nthreads=threads)
        c["search"] = pick(s, ANSWER + COUNTS)
        c["search_radius"] = rad
        e["opta"] = c
        save(db)
    if "opta_paper" not in e:
        op, c = conditioning(img, m, n, True, threads)
        s = O.opta_paper_search(img, op["image"], tpl, op["h"], op["w"], op["radius"], nthreads=threads)
        c["search"] = pick(s, ANSWER + ("n_locations", "n_centres", "n_eliminated", "n_survivors", "n_computed"))
        c["search_radius"] = op["radius"]
        e["opta_paper"] = c
        save(db)
    log(f"workload 2 done: {e['plain']}")


def do_workload3(db, threads):
    w = workload(3)
    img = w["images"][0]
    e = db.setdefault("3", {})
    e["image_sha256"] = sha(img)
    cond = e.setdefault("opta", {})
    Js = {}
    for size in sorted({t.shape[0] for t, _, _ in w["templates"]}):
        if str(size) in cond:
            continue
        log(f"workload 3: conditioning for {size}x{size}")
        op, c = conditioning(img, size, size, False, threads)
        Js[size] = op
        cond[str(size)] = c
        save(db)
    tl = e.setdefault("templates", [])
    for k, (tpl, loc, _) in enumerate(w["templates"]):
        if k < len(tl) and "opta_search" in tl[k]:
            continue
        m, n = tpl.shape
        log(f"workload 3: template {k} ({m}x{n})")
        rec = tl[k] if k < len(tl) else {}
        rec.update({"template_sha256": sha(tpl), "cut": list(loc), "size": [m, n]})
        if "plain" not in rec:
            rec["plain"] = plain(img, tpl, threads)
            if k >= len(tl):
                tl.append(rec)
            save(db)
        if m not in Js:
            Js[m] = O.opta(img, m, n, nthreads=threads)
            assert sha(Js[m]["image"]) == cond[str(m)]["image_sha256"]
        op = Js[m]
        rad = max(op["radius"], 2)
        s = O.opta_search(img, op["image"], tpl, op["h"], op["w"], rad, nthreads=threads)
        rec["opta_search"] = pick(s, ANSWER + COUNTS)
        rec["opta_search_radius"] = rad
        if k >= len(tl):
            tl.append(rec)
        save(db)
    log("workload 3 done")


def do_workload4(db, threads):
    w = workload(4)
    img = w["images"][0]
    e = db.setdefault("4", {})
    e["image_sha256"] = sha(img)
    tl = e.setdefault("templates", [])
    for k, (tpl, loc, _) in enumerate(w["templates"]):
        if k < len(tl):
            continue
        log(f"workload 4: template {k} {tpl.shape}")
        rec = {"template_sha256": sha(tpl), "cut": list(loc), "size": list(tpl.shape),
               "plain": plain(img, tpl, threads)}
        tl.append(rec)
        save(db)
    log("workload 4 done")


def do_workload5(db, threads):
    imgs = workload(5)["images"]
    e = db.setdefault("5", {})
    e["image_sha256"] = [sha(im) for im in imgs]
    e["queries"] = N_SERVE
    tl = e.setdefault("templates", [])
    qs = serving_queries(imgs, N_SERVE)
    for k, (tpl, j, loc) in enumerate(qs):
        if k < len(tl):
            continue
        log(f"workload 5: query {k} {tpl.shape} on image {j}")
        rec = {"template_sha256": sha(tpl), "image": j, "cut": list(loc) if loc else None,
               "size": list(tpl.shape), "plain": plain(imgs[j], tpl, threads)}
        tl.append(rec)
        save(db)
    log("workload 5 done")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--only", default="2,3,4,5")
    a = ap.parse_args()
    db = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for w in a.only.split(","):
        {"2": do_workload2, "3": do_workload3, "4": do_workload4, "5": do_workload5}[w](db, a.threads)


if __name__ == "__main__":
    main()
