// Host mirror of the device graph: two slotted CSR lists (in-lists by sink, out-lists by
// source) whose slot arrays match the device copies entry for entry. Every edit produces the
// device writes that keep the copies equal; rows that outgrow their slots move to the end of
// the slot array, and a full slot array is repacked and uploaded whole.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <unordered_set>
#include <vector>

namespace sr {

struct Write {
  int32_t array;  // 0 start, 1 len, 2 idx (per list; the caller adds the list's offset)
  int32_t index;
  int32_t value;
};

struct SlotList {
  std::vector<int32_t> start, len, cap;
  std::vector<int32_t> idx;
  std::vector<double> w;  // per slot weights (weighted graphs only)
  int64_t used = 0;
  int64_t need = 0;  // slots a repack would take now: sum over rows of packed_cap(len)
  bool weighted = false;

  static int32_t slack_cap(int32_t l) { return l + std::max<int32_t>(4, l / 4); }
  static int64_t packed_cap(int64_t l) { return l ? slack_cap((int32_t)l) : 0; }

  // Whether appending add[r] entries to each listed row r (rows ascending or not) is
  // guaranteed to succeed: a repack after all of them, plus one fresh row, fits the slot
  // array. Every insertion path (in place, row move, repack) succeeds when this holds.
  template <typename Map>
  bool fits(const Map& add) const {
    int64_t after = need;
    for (const auto& ra : add)
      after += packed_cap((int64_t)len[ra.first] + ra.second) - packed_cap(len[ra.first]);
    return after + 4 <= (int64_t)idx.size();
  }

  // Builds rows of nodes [0, node_cap) from (row, val) pairs in edge order.
  void build(int64_t node_cap, int64_t slot_cap, const std::vector<int32_t>& row,
             const std::vector<int32_t>& val, const double* wts) {
    start.assign(node_cap, 0);
    len.assign(node_cap, 0);
    cap.assign(node_cap, 0);
    for (int32_t r : row) len[r]++;
    int64_t pos = 0;
    for (int64_t r = 0; r < node_cap; ++r) {
      start[r] = (int32_t)pos;
      cap[r] = len[r] ? slack_cap(len[r]) : 0;
      pos += cap[r];
    }
    used = pos;
    need = pos;
    idx.assign(std::max<int64_t>(slot_cap, pos), -1);
    weighted = wts != nullptr;
    if (weighted) w.assign(idx.size(), 0.0);
    std::vector<int32_t> fill(node_cap, 0);
    for (size_t e = 0; e < row.size(); ++e) {
      const int32_t r = row[e];
      const int64_t p = start[r] + fill[r]++;
      idx[p] = val[e];
      if (weighted) w[p] = wts[e];
    }
  }

  // Rebuilds with fresh slack (row order preserved). Returns false if slot_cap is too small.
  bool repack() {
    int64_t tot = 0;
    for (size_t r = 0; r < len.size(); ++r) tot += packed_cap(len[r]);
    if (tot > (int64_t)idx.size()) return false;
    std::vector<int32_t> nidx(idx.size(), -1);
    std::vector<double> nw;
    if (weighted) nw.assign(idx.size(), 0.0);
    int64_t pos = 0;
    for (size_t r = 0; r < len.size(); ++r) {
      const int32_t c = len[r] ? slack_cap(len[r]) : 0;
      for (int32_t p = 0; p < len[r]; ++p) {
        nidx[pos + p] = idx[start[r] + p];
        if (weighted) nw[pos + p] = w[start[r] + p];
      }
      start[r] = (int32_t)pos;
      cap[r] = c;
      pos += c;
    }
    idx.swap(nidx);
    if (weighted) w.swap(nw);
    used = pos;
    need = pos;
    return true;
  }

  int32_t find(int32_t r, int32_t v) const {
    for (int32_t p = 0; p < len[r]; ++p)
      if (idx[start[r] + p] == v) return p;
    return -1;
  }

  // Appends v to row r. Returns 0 on an in-place edit (writes appended to out), 1 when the row
  // moved (its whole content must be uploaded: rows_moved gets r), 2 when the slot array was
  // repacked (the caller uploads everything), 3 when even a repack has no room: nothing is
  // appended (the rows may have been repacked, which the caller must upload). Callers check
  // fits() first, under which 3 does not occur.
  int insert(int32_t r, int32_t v, double wt, std::vector<Write>& out,
             std::vector<int32_t>& rows_moved) {
    const int rc = insert_impl(r, v, wt, out, rows_moved);
    if (rc != 3) need += packed_cap(len[r]) - packed_cap(len[r] - 1);
    return rc;
  }

  int insert_impl(int32_t r, int32_t v, double wt, std::vector<Write>& out,
                  std::vector<int32_t>& rows_moved) {
    if (len[r] < cap[r]) {
      const int32_t p = start[r] + len[r];
      idx[p] = v;
      if (weighted) w[p] = wt;
      len[r]++;
      out.push_back({2, p, v});
      out.push_back({1, r, len[r]});
      return 0;
    }
    const int32_t ncap = std::max<int32_t>(4, 2 * cap[r]);
    if (used + ncap > (int64_t)idx.size()) {
      // Slot array exhausted: repack every row with fresh slack, then append. The slot array
      // is sized so that a repack of any graph within the edge and node capacity fits and
      // leaves room for at least one more row allocation.
      if (!repack()) return 3;
      if (len[r] >= cap[r]) {
        if (used + 4 > (int64_t)idx.size()) return 3;
        start[r] = (int32_t)used;
        cap[r] = 4;
        used += 4;
      }
      const int32_t p = start[r] + len[r];
      idx[p] = v;
      if (weighted) w[p] = wt;
      len[r]++;
      return 2;
    }
    const int32_t ns = (int32_t)used;
    for (int32_t p = 0; p < len[r]; ++p) {
      idx[ns + p] = idx[start[r] + p];
      if (weighted) w[ns + p] = w[start[r] + p];
    }
    start[r] = ns;
    cap[r] = ncap;
    used += ncap;
    const int32_t p = start[r] + len[r];
    idx[p] = v;
    if (weighted) w[p] = wt;
    len[r]++;
    rows_moved.push_back(r);
    return 1;
  }

  // Removes v from row r by moving the row's last entry into its slot.
  bool remove(int32_t r, int32_t v, std::vector<Write>& out) {
    const int32_t p = find(r, v);
    if (p < 0) return false;
    const int32_t last = start[r] + len[r] - 1;
    const int32_t at = start[r] + p;
    if (at != last) {
      idx[at] = idx[last];
      if (weighted) w[at] = w[last];
      out.push_back({2, at, idx[at]});
    }
    idx[last] = -1;
    len[r]--;
    need += packed_cap(len[r]) - packed_cap(len[r] + 1);
    out.push_back({1, r, len[r]});
    return true;
  }
};

struct HostGraph {
  int64_t n = 0;
  int64_t m = 0;
  SlotList in;   // in-lists by sink: row j holds the sources i of edges i -> j
  SlotList out;  // out-lists by source: row i holds the sinks j of edges i -> j
  std::unordered_set<uint64_t> edges;

  static uint64_t key(int32_t i, int32_t j) {
    return ((uint64_t)(uint32_t)i << 32) | (uint32_t)j;
  }
  bool has(int32_t i, int32_t j) const { return edges.count(key(i, j)) != 0; }
};

}  // namespace sr
