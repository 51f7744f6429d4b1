#!/bin/bash
# Profile passes of bench.py on one MI355X: kernel trace with stats, HBM counters of
# the stencil kernels (FETCH_SIZE and WRITE_SIZE in passes of their own, scaled by the
# same counters of a plain 1 GiB device copy), vector-memory unit counters; then
# condense them into OUT/summary.md and OUT/stencil_traffic.json.
#
#     bash paper_1612_06424_amd/profile_bench.sh OUT
#
# Every pass launches the same kernel instances: DD_TUNE_CACHE names a copy of the
# stored launch shapes.  Each pass runs under its own time limit and the script stops
# at the first failing one.
set -u
R=$(cd "$(dirname "$0")/.." && pwd)
O=$(mkdir -p "$1" && cd "$1" && pwd)
rm -rf "$O"/trace "$O"/fetch "$O"/write "$O"/units "$O"/copy_fetch "$O"/copy_write
cp "$R"/paper_1612_06424_amd/tune_cache_mi355x.txt "$O"/tune_cache.txt
export DD_TUNE_CACHE=$O/tune_cache.txt
cd /tmp && export TMPDIR=/tmp
B=(--steps 1 --warmup 1 --no-cpu-baseline --parts stencil,solve,fact,batched,force)
SEL=(--kernel-include-regex "dslash|eo_hop|eo_lds")
echo "[profile] kernel trace"
timeout -s KILL 300 rocprofv3 --kernel-trace --stats -f csv -d "$O"/trace -o run -- python3 "$R"/bench.py "${B[@]}" > "$O"/trace.log 2>&1 || exit $?
find "$O"/trace -name "*kernel_trace.csv" -delete
echo "[profile] copy calibration"
timeout -s KILL 120 rocprofv3 --pmc FETCH_SIZE -f csv -d "$O"/copy_fetch -o run -- python3 "$R"/bench.py --copy-calibration > "$O"/copyf.log 2>&1 || exit $?
timeout -s KILL 120 rocprofv3 --pmc WRITE_SIZE -f csv -d "$O"/copy_write -o run -- python3 "$R"/bench.py --copy-calibration > "$O"/copyw.log 2>&1 || exit $?
echo "[profile] FETCH_SIZE"
timeout -s KILL 300 rocprofv3 --pmc FETCH_SIZE "${SEL[@]}" -f csv -d "$O"/fetch -o run -- python3 "$R"/bench.py "${B[@]}" > "$O"/fetch.log 2>&1 || exit $?
echo "[profile] WRITE_SIZE"
timeout -s KILL 300 rocprofv3 --pmc WRITE_SIZE "${SEL[@]}" -f csv -d "$O"/write -o run -- python3 "$R"/bench.py "${B[@]}" > "$O"/write.log 2>&1 || exit $?
echo "[profile] unit counters"
timeout -s KILL 300 rocprofv3 --pmc TA_TA_BUSY_sum TA_ADDR_STALLED_BY_TC_CYCLES_sum TCP_TCR_TCP_STALL_CYCLES_sum \
    TCP_PENDING_STALL_CYCLES_sum TCP_TOTAL_CACHE_ACCESSES_sum SQ_INSTS_VMEM_RD GRBM_GUI_ACTIVE "${SEL[@]}" \
    -f csv -d "$O"/units -o run -- python3 "$R"/bench.py "${B[@]}" > "$O"/units.log 2>&1 || exit $?
echo "[profile] summary"
cd "$R" && python3 -m paper_1612_06424_amd.rocprof_summary "$O" > "$O"/summary_print.log 2>&1 || exit $?
echo "[profile] done"
