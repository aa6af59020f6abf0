#!/bin/bash
# rocprofv3 passes over the evaluator and their summaries (run on a GPU machine).
#
#   paper_2603_12292_amd/profile.sh main OUTDIR PREFIX
#       kernel trace of the benchmark's main line, then one counter pass each
#       for FETCH_SIZE, WRITE_SIZE and SQ_INSTS_VALU + SQ_INSTS_SALU over
#       `profiling run` (benchmark workload + calibration copy); writes
#       PREFIX.txt and PREFIX_traffic.json
#   paper_2603_12292_amd/profile.sh paper|adjoint|ragged|loop OUTDIR PREFIX
#       kernel trace and counter passes (instruction mix, cycles and waits,
#       FETCH_SIZE, WRITE_SIZE) over the paper-regime evaluation, the
#       adjoint, the ragged batch or the paper's loop at 5e6 individuals;
#       writes PREFIX.txt and PREFIX.json (per-kernel means)
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
  bench_cmd="python3 bench.py --steps 20 --warmup 3 --main-only --no-ragged"
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
paper|adjoint|ragged|loop)
  # kernel trace plus two counter passes (instruction mix, then cycles and
  # waits) over the paper-regime evaluation (decode + resident interpreter)
  # or the adjoint of the differentiation workload
  if [ "$what" = paper ]; then
    run_cmd="python3 -m paper_2603_12292_amd.profiling paper --steps 2"
    kernels="k_prepare,k_eval_resident,k_eval_class,k_finalize,k_stage"
    title="paper regime: 2^20 programs (plain-mid x256, L~U{5..64}, D=5) on 512 cases, MSE"
  elif [ "$what" = loop ]; then
    run_cmd="python3 -m paper_2603_12292_amd.profiling loop --generations 3"
    kernels="k_generation,k_micro,k_init,k_prepare,k_eval_resident,k_eval_class,k_finalize,k_stage,k_target,k_values"
    title="paper loop: 5e6 individuals (ramped half-and-half, depths 2..5, max length 64, 9 base operators), correlation fitness on 512 cases (D=5), microcosm selection (sample 100, keep 0.5), mutation only; one untimed and 3 profiled generations"
  elif [ "$what" = ragged ]; then
    run_cmd="python3 -m paper_2603_12292_amd.profiling ragged --steps 2"
    kernels="k_eval_batch,k_prepare,k_stage,k_finalize,k_eval_class,k_eval_resident,k_target"
    title="ragged: 64 problems x 1024 programs, L~U{5..96}, D~U{1..9}, M=round(10^U(3,6)), MSE; batched (replayed graph), then one call per problem"
  else
    run_cmd="python3 -m paper_2603_12292_amd.profiling run --steps 2 --adjoint"
    kernels="k_grad,k_prepare,k_finalize"
    title="adjoint: N=4096 programs with 1..8 constants, L~U{8..64}, D=5, M=100000, MSE fitness and gradients"
  fi
  echo "pass: kernel trace"
  timeout -k 10 300 rocprofv3 --kernel-trace --stats --output-format csv -d "$out/trace" -- $run_cmd > "$out/trace.log"
  echo "pass: instruction mix"
  timeout -s KILL 120 rocprofv3 --pmc SQ_WAVES SQ_INSTS_VALU SQ_INSTS_SALU SQ_INSTS_LDS SQ_INSTS_VMEM SQ_INSTS_BRANCH \
    --output-format csv -d "$out/pmc_mix" -- $run_cmd > "$out/pmc_mix.log"
  echo "pass: cycles and waits"
  timeout -s KILL 120 rocprofv3 --pmc SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_WAIT_INST_LDS SQ_WAIT_ANY SQ_ACTIVE_INST_ANY \
    SQ_LDS_BANK_CONFLICT --output-format csv -d "$out/pmc_cyc" -- $run_cmd > "$out/pmc_cyc.log"
  echo "pass: FETCH_SIZE"
  timeout -s KILL 120 rocprofv3 --pmc FETCH_SIZE --output-format csv -d "$out/pmc_fetch" -- $run_cmd > "$out/pmc_fetch.log"
  echo "pass: WRITE_SIZE"
  timeout -s KILL 120 rocprofv3 --pmc WRITE_SIZE --output-format csv -d "$out/pmc_write" -- $run_cmd > "$out/pmc_write.log"
  python3 -m paper_2603_12292_amd.profiling summarize-kernels --trace "$out/trace" \
    --pmc "$out/pmc_mix" "$out/pmc_cyc" "$out/pmc_fetch" "$out/pmc_write" --kernels "$kernels" --out "$prefix" \
    --title "$title" \
    --command "paper_2603_12292_amd/profile.sh $what OUTDIR PREFIX (rocprofv3 --kernel-trace --stats -- $run_cmd; rocprofv3 --pmc SQ_WAVES SQ_INSTS_VALU SQ_INSTS_SALU SQ_INSTS_LDS SQ_INSTS_VMEM SQ_INSTS_BRANCH, then SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_WAIT_INST_LDS SQ_WAIT_ANY SQ_ACTIVE_INST_ANY SQ_LDS_BANK_CONFLICT, then FETCH_SIZE, then WRITE_SIZE -- $run_cmd)"
  ;;
*)
  echo "unknown pass set: $what" >&2
  exit 2
  ;;
esac
