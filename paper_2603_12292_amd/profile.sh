#!/bin/bash
# rocprofv3 passes over the evaluator and their summaries (run on a GPU machine).
#
#   paper_2603_12292_amd/profile.sh main OUTDIR PREFIX
#       kernel trace of the benchmark's main line, then one counter pass each
#       for FETCH_SIZE, WRITE_SIZE and SQ_INSTS_VALU + SQ_INSTS_SALU over
#       `profiling run` (benchmark workload + calibration copy); writes
#       PREFIX.txt and PREFIX_traffic.json
#   paper_2603_12292_amd/profile.sh ops OUTDIR PREFIX
#       SQ_INSTS_VALU + SQ_INSTS_SALU over `profiling ops` (single-operator
#       program shapes); writes PREFIX.txt
#
# Raw rocprofv3 output stays in OUTDIR; each pass runs under its own time
# limit and the script stops at the first failure.
set -euo pipefail
what=$1
mkdir -p "$2"
out=$(realpath "$2")
prefix=$(realpath -m "$3")
root=$(cd "$(dirname "$0")/.." && pwd)
export TMPDIR=/tmp
cd "$root"
case "$what" in
main)
  bench_cmd="python3 bench.py --steps 20 --warmup 3 --no-cpu-baseline --no-adjoint --no-ragged --no-scores --no-paper-shape --generations 0 --paper-loop 0"
  echo "pass: kernel trace"
  timeout -k 10 300 rocprofv3 --kernel-trace --stats --output-format csv -d "$out/trace" -- $bench_cmd > "$out/trace.log"
  for c in FETCH_SIZE WRITE_SIZE; do
    echo "pass: $c"
    timeout -s KILL 120 rocprofv3 --pmc $c --output-format csv -d "$out/pmc_$c" -- python3 -m paper_2603_12292_amd.profiling run > "$out/pmc_$c.log"
  done
  echo "pass: SQ_INSTS_VALU SQ_INSTS_SALU"
  timeout -s KILL 120 rocprofv3 --pmc SQ_INSTS_VALU SQ_INSTS_SALU --output-format csv -d "$out/pmc_SQ" -- python3 -m paper_2603_12292_amd.profiling run > "$out/pmc_SQ.log"
  python3 -m paper_2603_12292_amd.profiling summarize --trace "$out/trace" --fetch "$out/pmc_FETCH_SIZE" \
    --write "$out/pmc_WRITE_SIZE" --valu "$out/pmc_SQ" --out "$prefix" \
    --command "paper_2603_12292_amd/profile.sh main OUTDIR PREFIX (rocprofv3 --kernel-trace --stats -- $bench_cmd; rocprofv3 --pmc FETCH_SIZE, then WRITE_SIZE, then SQ_INSTS_VALU SQ_INSTS_SALU -- python3 -m paper_2603_12292_amd.profiling run)"
  ;;
ops)
  echo "pass: SQ_INSTS_VALU SQ_INSTS_SALU over the operator shapes"
  timeout -s KILL 120 rocprofv3 --pmc SQ_INSTS_VALU SQ_INSTS_SALU --output-format csv -d "$out/pmc_ops" -- python3 -m paper_2603_12292_amd.profiling ops > "$out/pmc_ops.log"
  python3 -m paper_2603_12292_amd.profiling summarize-ops --pmc "$out/pmc_ops" --out "$prefix" \
    --command "paper_2603_12292_amd/profile.sh ops OUTDIR PREFIX (rocprofv3 --pmc SQ_INSTS_VALU SQ_INSTS_SALU -- python3 -m paper_2603_12292_amd.profiling ops)"
  ;;
*)
  echo "unknown pass set: $what" >&2
  exit 2
  ;;
esac
