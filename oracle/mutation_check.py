"""Mutation check of the oracle's pins (test infrastructure).

Copies the repository to a temporary directory, plants one plausible mistake at
a time in oracle/orc.c (a flipped sign, a dropped term, a wrong index or
inequality), and runs tests/test_oracle_pins.py against the mutant.  Every
mutant must make at least one pin fail.  Usage: python oracle/mutation_check.py
"""
import os, shutil, subprocess, sys, tempfile
SRC = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
MUT = [
 ("dashpot sign", "double fm = p->kn * delta - p->gamma_n * vn;", "double fm = p->kn * delta + p->gamma_n * vn;"),
 ("normal flipped", "double nrm[3] = {(xi[0] - xj[0]) / d, (xi[1] - xj[1]) / d, (xi[2] - xj[2]) / d};", "double nrm[3] = {(xj[0] - xi[0]) / d, (xj[1] - xi[1]) / d, (xj[2] - xi[2]) / d};"),
 ("full kick at first half", "vfull[a] = (step == 0 && !p->v_in_is_half_step) ? vh[3 * i + a] : vh[3 * i + a] + hdt * acc;", "vfull[a] = (step == 0 && !p->v_in_is_half_step) ? vh[3 * i + a] : vh[3 * i + a] + p->dt * acc;"),
 ("skin without dt", "skin = p->K * norm3(v + 3 * i) * p->dt;", "skin = p->K * norm3(v + 3 * i);"),
 ("no cap", "rnl[i] = r < cap ? r : cap;", "rnl[i] = r;"),
 ("validity >=", "if (disp > skin_test[i]) viol++;", "if (disp >= skin_test[i]) viol++;"),
 ("skip same cell", "if (cb == ca && pb >= pa) continue;", "if (cb == ca) continue;"),
 ("hi wall sign", "if (dhi > 0.0) f[ax] -= p->kn * dhi - p->gamma_n * (-vi[ax]);", "if (dhi > 0.0) f[ax] += p->kn * dhi - p->gamma_n * (-vi[ax]);"),
 ("contact >=", "if (overlap(x + 3 * i, x + 3 * j, rc[i], rc[j]) > 0.0) pv_push(Ct, i, j);", "if (overlap(x + 3 * i, x + 3 * j, rc[i], rc[j]) >= 0.0) pv_push(Ct, i, j);"),
 ("drift with vfull", "x[3 * i + a] = x[3 * i + a] + p->dt * vh[3 * i + a];", "x[3 * i + a] = x[3 * i + a] + p->dt * vfull[a];"),
 ("x0 not refreshed", "memcpy(x0, x, n3 * sizeof(double));", ";"),
 ("damping uses vi only", "double vn = (vi[0] - vj[0]) * nrm[0] + (vi[1] - vj[1]) * nrm[1] + (vi[2] - vj[2]) * nrm[2];", "double vn = (vi[0]) * nrm[0] + (vi[1]) * nrm[1] + (vi[2]) * nrm[2];"),
 ("gravity dropped", "double acc = F[3 * i + a] * invm[i] + p->g[a];", "double acc = F[3 * i + a] * invm[i];"),
 ("invm ignored", "double acc = F[3 * i + a] * invm[i] + p->g[a];", "double acc = F[3 * i + a] + p->g[a];"),
 ("cell ring off by one", "for (int64_t dz = -ring; dz <= ring; dz++)", "for (int64_t dz = -ring + 1; dz <= ring; dz++)"),
 ("broad brute strict", "if (dist3(x + 3 * i, x + 3 * j) <= r[i] + r[j] + eps) pv_push(out, (int32_t)i, (int32_t)j);", "if (dist3(x + 3 * i, x + 3 * j) < r[i] + r[j] + eps) pv_push(out, (int32_t)i, (int32_t)j);"),
 ("skin from speed squared", "static double norm3(const double *a) { return sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]); }", "static double norm3(const double *a) { return (a[0] * a[0] + a[1] * a[1] + a[2] * a[2]); }"),
 ("eps dropped in linked cell", "if (dist3(x + 3 * pa, x + 3 * pb) <= r[pa] + r[pb] + eps) {", "if (dist3(x + 3 * pa, x + 3 * pb) <= r[pa] + r[pb]) {"),
 ("plane force reversed", "        f[0] += fm * pl[0];", "        f[0] -= fm * pl[0];"),
 ("plane offset sign", "double s = pl[0] * xi[0] + pl[1] * xi[1] + pl[2] * xi[2] - pl[3];", "double s = pl[0] * xi[0] + pl[1] * xi[1] + pl[2] * xi[2] + pl[3];"),
 ("plane height ignored", "if (!(xi[2] > pl[4])) continue;", ";"),
 ("friction opposes nothing", "          ft[c] = -p->kt * s[c] - p->gamma_t * vt[c];", "          ft[c] = p->kt * s[c] - p->gamma_t * vt[c];"),
 ("friction uncapped", "        if (ftn > lim) {", "        if (ftn > 1e300) {"),
 ("friction history dropped", "          for (int c = 0; c < 3; c++) s[c] = old->xi[3 * h + c];", "          ;"),
 ("friction tangent not projected", "          s[c] = (s[c] - sn * nrm[c]) + vt[c] * p->dt;", "          s[c] = s[c] + vt[c] * p->dt;"),
 ("plane damping sign", "double fm = p->kn * delta - p->gamma_n * vn;\n        f[0] += fm * pl[0];", "double fm = p->kn * delta + p->gamma_n * vn;\n        f[0] += fm * pl[0];"),
 ("kinetic energy of the half-step velocity", "kin[i] = 0.5 * (vfull[0] * vfull[0] + vfull[1] * vfull[1] + vfull[2] * vfull[2]) / invm[i];", "kin[i] = 0.5 * (vh[3 * i] * vh[3 * i] + vh[3 * i + 1] * vh[3 * i + 1] + vh[3 * i + 2] * vh[3 * i + 2]) / invm[i];"),
 ("kinetic energy without 1/2", "kin[i] = 0.5 * (vfull[0] * vfull[0]", "kin[i] = (vfull[0] * vfull[0]"),
 ("max_excess without the skin", "double excess = disp - skin_test[i];", "double excess = disp;"),
 ("list_pairs as contact count", "r->list_pairs = p->skin_mode == ORC_NAIVE ? 0 : list_pairs;", "r->list_pairs = p->skin_mode == ORC_NAIVE ? 0 : C.n;"),
 ("violators off by one", "if (disp > skin_test[i]) viol++;", "if (disp > skin_test[i]) viol += 2;"),
 ("cylinder normal outward", "double nx = -ex / rho;\n        double ny = -ey / rho;", "double nx = ex / rho;\n        double ny = ey / rho;"),
 ("cylinder overlap outside the wall", "double delta = rc[i] - (cyl[2] - rho);", "double delta = rc[i] - (cyl[2] + rho);"),
 ("cylinder height ignored", "if (!(xi[2] > cyl[3])) continue;", ";"),
 ("cylinder damping sign", "double fm = p->kn * delta - p->gamma_n * vn;\n        f[0] += fm * nx;", "double fm = p->kn * delta + p->gamma_n * vn;\n        f[0] += fm * nx;"),
 ("cylinder y force dropped", "        f[1] += fm * ny;", "        ;"),
 ("lo wall damping sign", "if (dlo > 0.0) f[ax] += p->kn * dlo - p->gamma_n * vi[ax];", "if (dlo > 0.0) f[ax] += p->kn * dlo + p->gamma_n * vi[ax];"),
 ("friction spring without dt", "s[c] = (s[c] - sn * nrm[c]) + vt[c] * p->dt;", "s[c] = (s[c] - sn * nrm[c]) + vt[c];"),
 ("tangential dashpot dropped", "ft[c] = -p->kt * s[c] - p->gamma_t * vt[c];", "ft[c] = -p->kt * s[c];"),
 ("cone on |F_n|", "double lim = p->mu * (fm > 0.0 ? fm : 0.0);", "double lim = p->mu * fabs(fm);"),
 ("sliding spring kept", "s[c] = p->kt > 0.0 ? -(ft[c] + p->gamma_t * vt[c]) / p->kt : 0.0;", "s[c] = s[c];"),
 ("sliding spring without dashpot part", "s[c] = p->kt > 0.0 ? -(ft[c] + p->gamma_t * vt[c]) / p->kt : 0.0;", "s[c] = p->kt > 0.0 ? -ft[c] / p->kt : 0.0;"),
 ("history lookup past the partner", "while (h < h_end && old->j[h] < j) h++;", "while (h < h_end && old->j[h] <= j) h++;"),
 ("fixed interval offset", "rebuild = (step % p->fixed_interval) == 0;", "rebuild = ((step + 1) % p->fixed_interval) == 0;"),
 ("uniform skin from K", "case ORC_FIXED_INTERVAL: skin = p->skin_uniform; break;", "case ORC_FIXED_INTERVAL: skin = p->K * norm3(v + 3 * i) * p->dt; break;"),
 ("force overlap from own radius", "double delta = rc[i] + rc[j] - d;", "double delta = 2.0 * rc[i] - d;"),
 ("contact test from own radius", "  return ri + rj - dist3(xi, xj);", "  return 2.0 * ri - dist3(xi, xj);"),
 ("broad phase from own radius", "if (dist3(x + 3 * pa, x + 3 * pb) <= r[pa] + r[pb] + eps) {", "if (dist3(x + 3 * pa, x + 3 * pb) <= 2.0 * r[pa] + eps) {"),
 ("no rebuild at step 0", "else rebuild = (step == 0) || violated;", "else rebuild = violated;"),
 ("second half-kick dropped", "vh[3 * i + a] = vfull[a] + hdt * acc;", "vh[3 * i + a] = vfull[a];"),
 ("displacement from the current position", "double disp = dist3(x + 3 * i, x0 + 3 * i);", "double disp = dist3(x + 3 * i, x + 3 * i);"),
 ("plane distance without offset", "double s = pl[0] * xi[0] + pl[1] * xi[1] + pl[2] * xi[2] - pl[3];", "double s = pl[0] * xi[0] + pl[1] * xi[1] + pl[2] * xi[2];"),
]
dst = os.path.join(tempfile.mkdtemp(prefix='orc_mut_'), 'repo')
results = []
survivors = 0
for name, a, b in MUT:
    if os.path.exists(dst): shutil.rmtree(os.path.dirname(dst))
    shutil.copytree(SRC, dst, ignore=shutil.ignore_patterns('.git', '_work', '*_out', '*.so', '__pycache__'))
    p = os.path.join(dst, 'oracle/orc.c')
    s = open(p).read()
    assert a in s, name
    open(p, 'w').write(s.replace(a, b, 1))
    # the pattern test fails on any mutant (its target text is gone): the pins alone must catch it
    r = subprocess.run([sys.executable, '-m', 'pytest', '-q', '-x', 'tests/test_oracle_pins.py', '-p', 'no:cacheprovider',
                        '--deselect', 'tests/test_oracle_pins.py::test_mutation_check_patterns_match_the_oracle'],
                       cwd=dst, capture_output=True, text=True)
    last = [l for l in r.stdout.splitlines() if 'failed' in l or 'passed' in l][-1:]
    results.append((name, r.returncode != 0, last))
    survivors += r.returncode == 0
    print(f"{name:28s} {'CAUGHT' if r.returncode else 'SURVIVED'} {last}", flush=True)
shutil.rmtree(os.path.dirname(dst))
sys.exit(1 if survivors else 0)
