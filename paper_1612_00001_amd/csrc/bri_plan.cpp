// Host planner: turns the recursive Schur complement splitting into a list of
// batched steps over b x b workspace slots.
//
// Notation (principal elimination order): v(r, c, I) is block (r, c) after the
// blocks in I were eliminated,
//     v(r, c, I) = v(r, c, I') - v(r, p, I') v(p, p, I')^{-1} v(p, c, I'),
// p the last entry of I (the Schur complement of eqs. SchurofA..SchurofD with
// the pivot moved to the principal position).  A node of depth d has the four
// children (r,c), (r,p), (p,p), (p,c) of depth d-1; depth-0 nodes are blocks of
// M.  The recursion recomputes every child, as the backward procedure of the
// paper does branch by branch (Section "Implementation"), so one block costs
// sum_{i=1}^{k-1} 4^{k-1-i} Schur operations (Theorem "C_BRI").
//
// Evaluation order.  Nodes of one depth are processed in lock-step batches of
// at most W (the largest power of 4 not above W): for a batch of nodes the planner evaluates all their pivot
// children, factors them, evaluates the right-hand children and solves, then
// the left children (accumulated into one running sum per chain), and finally
// the diagonal children, whose last product subtracts the accumulated sum.
// Each recursion level holds one pending block per node of the batch, which
// keeps the live workspace at about (depth + 3) blocks per batch entry
// (Theorem "MC_BRI" bounds it by O(b^2) per branch); with W = 1 the peak is
// (k + 1) blocks.  Result blocks are allocated only when they are written.
// Above the depth at which a level reaches W nodes the tree is expanded
// breadth first.
#include <algorithm>
#include <cmath>
#include <stdexcept>

#include "bri_internal.h"

namespace bri {

namespace {

struct SlotPool {
  std::vector<int> free_list;
  int next = 0;
  int live = 0;
  int peak = 0;
  int alloc() {
    int s;
    if (!free_list.empty()) {
      s = free_list.back();
      free_list.pop_back();
    } else {
      s = next++;
    }
    ++live;
    peak = std::max(peak, live);
    return s;
  }
  void release(int s) {
    free_list.push_back(s);
    --live;
  }
};

// A node of the recursion: (r, c) at depth d in the principal order, or
// frame f (depth = its size - 1) of the paper's literal frame procedure.
struct Node {
  int r, c, depth;
  int f = -1;
};

// The frames of the paper's forward procedure (Section "Forward recursive
// procedure"), for the literal elimination order.  A frame is a list of
// block rows and one of block columns with a type (R for the root, else the
// child position A, B, C or D it came from).  A frame of at least three
// blocks a side first exchanges its two leading block columns (types B, D)
// and / or rows (types C, D), so that the block its parent regarded as M_22
// is back at position (2, 2); then its children drop the last row and
// column (A), the last row and first column (B), the first row and last
// column (C), or the first row and column (D).  Frames of two blocks a side
// are the leaves: their four blocks are blocks of M.
struct LitFrame {
  std::vector<int> rows, cols;
  char type;
  int kid[4];  // child frames A, B, C, D (-1 for a leaf frame)
};

class LitTree {
 public:
  // Root frame of block (i, j): block rows 0 and j and block columns 0 and
  // i exchanged, so that N_ij is the (1, 1) block of the permuted inverse.
  LitTree(int k, int i, int j) {
    std::vector<int> rows(k), cols(k);
    for (int t = 0; t < k; ++t) rows[t] = cols[t] = t;
    std::swap(rows[0], rows[j]);
    std::swap(cols[0], cols[i]);
    root_ = visit(rows, cols, 'R');
  }
  int root() const { return root_; }
  const LitFrame& at(int f) const { return frames_[f]; }
  // Positions (A, B, C, D = 0..3) of the operands X, Y, Z, W of the frame's
  // Schur complement X - Y Z^{-1} W for its type: the root and A frames
  // take (M/D) = A - B D^{-1} C, B frames (M/C) = B - A C^{-1} D, C frames
  // (M/B) = C - D B^{-1} A and D frames (M/A) = D - C A^{-1} B (eqs.
  // SchurofD, SchurofC, SchurofB, SchurofA).
  static void roles(char type, int& x, int& y, int& z, int& w) {
    switch (type) {
      case 'B': x = 1; y = 0; z = 2; w = 3; break;
      case 'C': x = 2; y = 3; z = 1; w = 0; break;
      case 'D': x = 3; y = 2; z = 0; w = 1; break;
      default:  x = 0; y = 1; z = 3; w = 2; break;
    }
  }

 private:
  int visit(std::vector<int> rows, std::vector<int> cols, char type) {
    const size_t m = rows.size();
    if (m >= 3) {
      if (type == 'B' || type == 'D') std::swap(cols[0], cols[1]);
      if (type == 'C' || type == 'D') std::swap(rows[0], rows[1]);
    }
    const int id = static_cast<int>(frames_.size());
    frames_.push_back(LitFrame{rows, cols, type, {-1, -1, -1, -1}});
    if (m >= 3) {
      const std::vector<int> r_head(rows.begin(), rows.end() - 1), r_tail(rows.begin() + 1, rows.end());
      const std::vector<int> c_head(cols.begin(), cols.end() - 1), c_tail(cols.begin() + 1, cols.end());
      const int a = visit(r_head, c_head, 'A');
      const int b = visit(r_head, c_tail, 'B');
      const int c = visit(r_tail, c_head, 'C');
      const int d = visit(r_tail, c_tail, 'D');
      frames_[id].kid[0] = a;
      frames_[id].kid[1] = b;
      frames_[id].kid[2] = c;
      frames_[id].kid[3] = d;
    }
    return id;
  }
  std::vector<LitFrame> frames_;
  int root_ = -1;
};

class Builder {
 public:
  Builder(Plan& p, std::vector<int> elim, int width) : plan_(p), elim_(std::move(elim)), width_(width) {}
  // Literal frame order: nodes are frames of tree t (which must outlive the
  // builder) and carry their own operand roles.
  void set_literal(const LitTree* t) { lit_ = t; }

  // The children of node u in the roles of its Schur complement
  // X - Y Z^{-1} W (principal order: X = (r, c), Y = (r, p), Z = (p, p),
  // W = (p, c) at depth d - 1, p the pivot of depth d).
  void kids_of(const Node& u, Node& x, Node& y, Node& z, Node& w) const {
    if (lit_) {
      const LitFrame& F = lit_->at(u.f);
      int rx, ry, rz, rw;
      LitTree::roles(F.type, rx, ry, rz, rw);
      x = Node{-1, -1, u.depth - 1, F.kid[rx]};
      y = Node{-1, -1, u.depth - 1, F.kid[ry]};
      z = Node{-1, -1, u.depth - 1, F.kid[rz]};
      w = Node{-1, -1, u.depth - 1, F.kid[rw]};
      return;
    }
    const int p = pivot_of(u.depth);
    x = Node{u.r, u.c, u.depth - 1};
    y = Node{u.r, p, u.depth - 1};
    z = Node{p, p, u.depth - 1};
    w = Node{p, u.c, u.depth - 1};
  }
  // The blocks of a depth-1 node in the same roles (W and X may stand for
  // the right-hand side column of a solve plan).
  void leaf_blocks(const Node& u, Opnd& x, Opnd& y, Opnd& z, Opnd& w) const {
    if (lit_) {
      const LitFrame& F = lit_->at(u.f);
      const Opnd q[4] = {Opnd::mblk(F.rows[0], F.cols[0]), Opnd::mblk(F.rows[0], F.cols[1]),
                         Opnd::mblk(F.rows[1], F.cols[0]), Opnd::mblk(F.rows[1], F.cols[1])};
      int rx, ry, rz, rw;
      LitTree::roles(F.type, rx, ry, rz, rw);
      x = q[rx];
      y = q[ry];
      z = q[rz];
      w = q[rw];
      return;
    }
    const int p = pivot_of(1);
    x = blk(u.r, u.c);
    y = Opnd::mblk(u.r, p);
    z = Opnd::mblk(p, p);
    w = blk(p, u.c);
  }

  int next_node() { return node_counter_++; }
  SlotPool& pool() { return pool_; }

  // Block column index standing for the right-hand side R of a solve plan.
  void set_rhs_column(int c) { rhs_col_ = c; }
  // Pivot memo: memo[d - 1] is a slot holding the already factored and
  // inverted pivot v(p, p, I') of every depth-d node (p = pivot_of(d)), or -1.
  // Memoised pivots are neither recomputed nor refactored: a node then has
  // three children instead of four.
  void set_memo(std::vector<int> memo) { memo_ = std::move(memo); }

  // Depth-0 operand (r, c): a block of Gamma, or of R for the RHS column.
  Opnd blk(int r, int c) const { return c == rhs_col_ ? Opnd::rhs(r) : Opnd::mblk(r, c); }
  int memo_of(int depth) const {
    return depth - 1 < static_cast<int>(memo_.size()) ? memo_[depth - 1] : -1;
  }

  Step& step(StepKind kind) {
    plan_.steps.push_back(Step{kind, {}});
    return plan_.steps.back();
  }

  // Evaluates the batch L (all of one depth d >= 1) and returns the slots
  // holding the results (allocated only when the result is written); when
  // accs[t] >= 0 the accumulated sum in that slot is subtracted at the end.
  std::vector<int> eval(const std::vector<Node>& L, const std::vector<int>& accs) {
    if (L.empty()) return {};
    const int d = L[0].depth;
    if (d == 1) return leaf(L, accs);
    const int64_t kids = memo_of(d) >= 0 ? 3 : 4;
    if (kids * static_cast<int64_t>(L.size()) <= width_) return expand(L, accs);
    return lockstep(L, accs);
  }

  // X = P^{-1} B with already inverted factors: lu[t] holds the factors,
  // rhs[t] the operand B, xdst[t] receives X.  One Schur operation each.
  void solve_with(const std::vector<int>& lu, const std::vector<Opnd>& rhs, const std::vector<Opnd>& xdst) {
    const size_t n = lu.size();
    std::vector<int> tmp(n);
    for (size_t t = 0; t < n; ++t) tmp[t] = pool_.alloc();
    Step& l = step(ST_TRMM_L);
    for (size_t t = 0; t < n; ++t) {
      StepItem it;
      it.dst = Opnd::slot(tmp[t]);
      it.x = Opnd::slot(lu[t]);
      it.y = rhs[t];
      l.items.push_back(it);
    }
    Step& u = step(ST_TRMM_U);
    for (size_t t = 0; t < n; ++t) {
      StepItem it;
      it.dst = xdst[t];
      it.x = Opnd::slot(lu[t]);
      it.y = Opnd::slot(tmp[t]);
      u.items.push_back(it);
    }
    for (size_t t = 0; t < n; ++t) pool_.release(tmp[t]);
  }

  // Factor pivots, invert their triangular factors and form X = P^{-1} B for
  // a batch; lu[t] holds the pivot, rhs[t] the operand B; the result X goes to
  // xdst[t].  Releases nothing.
  void factor_and_solve(const std::vector<int>& lu, const std::vector<Opnd>& rhs, const std::vector<Opnd>& xdst,
                        bool count_schur) {
    const size_t n = lu.size();
    // The scratch block of the triangular inversion is also the shadow of
    // the recursive LU, so it is taken before the factorisation.
    std::vector<int> tmp(n);
    for (size_t t = 0; t < n; ++t) tmp[t] = pool_.alloc();
    Step& g = step(ST_GETRF);
    for (size_t t = 0; t < n; ++t) {
      StepItem it;
      it.dst = Opnd::slot(lu[t]);
      it.x = Opnd::slot(tmp[t]);
      it.node = next_node();
      g.items.push_back(it);
      if (count_schur) plan_.schur_ops++;
    }
    Step& tr = step(ST_TRTRI);
    for (size_t t = 0; t < n; ++t) {
      StepItem it;
      it.dst = Opnd::slot(lu[t]);
      it.x = Opnd::slot(tmp[t]);
      tr.items.push_back(it);
    }
    Step& l = step(ST_TRMM_L);
    for (size_t t = 0; t < n; ++t) {
      StepItem it;
      it.dst = Opnd::slot(tmp[t]);
      it.x = Opnd::slot(lu[t]);
      it.y = rhs[t];
      l.items.push_back(it);
    }
    Step& u = step(ST_TRMM_U);
    for (size_t t = 0; t < n; ++t) {
      StepItem it;
      it.dst = xdst[t];
      it.x = Opnd::slot(lu[t]);
      it.y = Opnd::slot(tmp[t]);
      u.items.push_back(it);
    }
    for (size_t t = 0; t < n; ++t) pool_.release(tmp[t]);
  }

  int pivot_of(int depth) const { return elim_[depth - 1]; }

 private:
  std::vector<int> leaf(const std::vector<Node>& L, const std::vector<int>& accs) {
    const size_t n = L.size();
    const int memo = memo_of(1);
    std::vector<int> sp(n), sx(n), outs(n);
    std::vector<Opnd> rhs(n), xd(n), bx(n), by(n), bz(n);
    for (size_t t = 0; t < n; ++t) {
      leaf_blocks(L[t], bx[t], by[t], bz[t], rhs[t]);
    }
    if (memo >= 0) {
      for (size_t t = 0; t < n; ++t) sx[t] = pool_.alloc();
      for (size_t t = 0; t < n; ++t) xd[t] = Opnd::slot(sx[t]);
      solve_with(std::vector<int>(n, memo), rhs, xd);
      plan_.schur_ops += static_cast<int64_t>(n);
    } else {
      for (size_t t = 0; t < n; ++t) sp[t] = pool_.alloc();
      for (size_t t = 0; t < n; ++t) sx[t] = pool_.alloc();
      Step& ld = step(ST_LOAD);
      for (size_t t = 0; t < n; ++t) {
        StepItem it;
        it.dst = Opnd::slot(sp[t]);
        it.x = bz[t];
        ld.items.push_back(it);
      }
      for (size_t t = 0; t < n; ++t) xd[t] = Opnd::slot(sx[t]);
      factor_and_solve(sp, rhs, xd, true);
      for (size_t t = 0; t < n; ++t) pool_.release(sp[t]);
    }
    for (size_t t = 0; t < n; ++t) outs[t] = pool_.alloc();
    Step& g = step(ST_GEMM);
    for (size_t t = 0; t < n; ++t) {
      StepItem it;
      it.dst = Opnd::slot(outs[t]);
      it.x = by[t];
      it.y = Opnd::slot(sx[t]);
      it.cin = bx[t];
      it.sub = accs[t] >= 0 ? Opnd::slot(accs[t]) : Opnd::none();
      g.items.push_back(it);
    }
    for (size_t t = 0; t < n; ++t) pool_.release(sx[t]);
    return outs;
  }

  std::vector<int> expand(const std::vector<Node>& L, const std::vector<int>& accs) {
    const size_t n = L.size();
    const int d = L[0].depth;
    const int memo = memo_of(d);
    const int nk = memo >= 0 ? 3 : 4;
    std::vector<Node> kids;
    for (size_t t = 0; t < n; ++t) {
      Node x, y, z, w;
      kids_of(L[t], x, y, z, w);
      kids.push_back(x);
      kids.push_back(y);
      if (memo < 0) kids.push_back(z);
      kids.push_back(w);
    }
    const std::vector<int> res = eval_children(kids);
    std::vector<int> src(n), srp(n), spp(n), spc(n);
    for (size_t t = 0; t < n; ++t) {
      src[t] = res[nk * t];
      srp[t] = res[nk * t + 1];
      spp[t] = memo >= 0 ? memo : res[nk * t + 2];
      spc[t] = res[nk * t + nk - 1];
    }
    std::vector<Opnd> rhs(n), xd(n);
    for (size_t t = 0; t < n; ++t) {
      rhs[t] = Opnd::slot(spc[t]);
      xd[t] = Opnd::slot(spc[t]);
    }
    if (memo >= 0) {
      solve_with(spp, rhs, xd);
      plan_.schur_ops += static_cast<int64_t>(n);
    } else {
      factor_and_solve(spp, rhs, xd, true);
      for (size_t t = 0; t < n; ++t) pool_.release(spp[t]);
    }
    Step& g = step(ST_GEMM);
    for (size_t t = 0; t < n; ++t) {
      StepItem it;
      it.dst = Opnd::slot(src[t]);
      it.x = Opnd::slot(srp[t]);
      it.y = Opnd::slot(spc[t]);
      it.cin = Opnd::slot(src[t]);
      it.sub = accs[t] >= 0 ? Opnd::slot(accs[t]) : Opnd::none();
      g.items.push_back(it);
    }
    for (size_t t = 0; t < n; ++t) {
      pool_.release(srp[t]);
      pool_.release(spc[t]);
    }
    return src;
  }

  std::vector<int> lockstep(const std::vector<Node>& L, const std::vector<int>& accs) {
    const size_t n = L.size();
    const int d = L[0].depth;
    const int memo = memo_of(d);
    const std::vector<int> none(n, -1);
    std::vector<Node> kx(n), ky(n), kz(n), kw(n);
    for (size_t t = 0; t < n; ++t) kids_of(L[t], kx[t], ky[t], kz[t], kw[t]);
    std::vector<Node> kids(n);
    std::vector<int> sp(n, memo);
    if (memo < 0) {
      // Pivot children, factored at once so only their factors stay live.
      kids = kz;
      sp = eval_children(kids);
      factor_only(sp);
    }
    // Right-hand children; X = P^{-1} B replaces them.
    kids = kw;
    const std::vector<int> sb = eval_children(kids);
    if (memo < 0) {
      solve_only(sp, sb);
      for (size_t t = 0; t < n; ++t) pool_.release(sp[t]);
    } else {
      std::vector<Opnd> ob(n);
      for (size_t t = 0; t < n; ++t) ob[t] = Opnd::slot(sb[t]);
      solve_with(sp, ob, ob);
      plan_.schur_ops += static_cast<int64_t>(n);
    }
    // Left children: acc (+)= C X.
    kids = ky;
    const std::vector<int> sc = eval_children(kids);
    std::vector<int> acc(n);
    std::vector<bool> own(n, false);
    for (size_t t = 0; t < n; ++t) {
      if (accs[t] >= 0) {
        acc[t] = accs[t];
      } else {
        acc[t] = pool_.alloc();
        own[t] = true;
      }
    }
    Step& g = step(ST_GEMM_ACC);
    for (size_t t = 0; t < n; ++t) {
      StepItem it;
      it.dst = Opnd::slot(acc[t]);
      it.x = Opnd::slot(sc[t]);
      it.y = Opnd::slot(sb[t]);
      it.cin = own[t] ? Opnd::none() : Opnd::slot(acc[t]);
      g.items.push_back(it);
    }
    for (size_t t = 0; t < n; ++t) {
      pool_.release(sc[t]);
      pool_.release(sb[t]);
    }
    // Diagonal children subtract the accumulated sum in their last product.
    kids = kx;
    const std::vector<int> outs = eval_children(kids, acc);
    for (size_t t = 0; t < n; ++t)
      if (own[t]) pool_.release(acc[t]);
    return outs;
  }

 public:
  void factor_only(const std::vector<int>& lu) {
    std::vector<int> tmp;
    for (size_t t = 0; t < lu.size(); ++t) tmp.push_back(pool_.alloc());
    Step& g = step(ST_GETRF);
    for (size_t t = 0; t < lu.size(); ++t) {
      StepItem it;
      it.dst = Opnd::slot(lu[t]);
      it.x = Opnd::slot(tmp[t]);
      it.node = next_node();
      g.items.push_back(it);
      plan_.schur_ops++;
    }
    Step& tr = step(ST_TRTRI);
    for (size_t t = 0; t < lu.size(); ++t) {
      StepItem it;
      it.dst = Opnd::slot(lu[t]);
      it.x = Opnd::slot(tmp[t]);
      tr.items.push_back(it);
    }
    for (int s : tmp) pool_.release(s);
  }

  // X = U^{-1} L^{-1} P B in place of B (lu already holds the inverted factors).
  void solve_only(const std::vector<int>& lu, const std::vector<int>& b) {
    std::vector<int> tmp;
    for (size_t t = 0; t < lu.size(); ++t) tmp.push_back(pool_.alloc());
    Step& l = step(ST_TRMM_L);
    for (size_t t = 0; t < lu.size(); ++t) {
      StepItem it;
      it.dst = Opnd::slot(tmp[t]);
      it.x = Opnd::slot(lu[t]);
      it.y = Opnd::slot(b[t]);
      l.items.push_back(it);
    }
    Step& u = step(ST_TRMM_U);
    for (size_t t = 0; t < lu.size(); ++t) {
      StepItem it;
      it.dst = Opnd::slot(b[t]);
      it.x = Opnd::slot(lu[t]);
      it.y = Opnd::slot(tmp[t]);
      u.items.push_back(it);
    }
    for (int s : tmp) pool_.release(s);
  }

  // Inverse of the matrix in slot z written to dst: getrf, triangular
  // inversion, then U^{-1} (L^{-1} P I).
  void final_inverse(int z, Opnd dst, bool count_final) {
    int tmp = pool_.alloc();
    Step& g = step(ST_GETRF);
    StepItem it;
    it.dst = Opnd::slot(z);
    it.x = Opnd::slot(tmp);
    it.node = next_node();
    g.items.push_back(it);
    if (count_final) plan_.final_inversions++;
    Step& tr = step(ST_TRTRI);
    StepItem t1;
    t1.dst = Opnd::slot(z);
    t1.x = Opnd::slot(tmp);
    tr.items.push_back(t1);
    Step& l = step(ST_TRMM_L);
    StepItem t2;
    t2.dst = Opnd::slot(tmp);
    t2.x = Opnd::slot(z);
    t2.y = Opnd::ident();
    l.items.push_back(t2);
    Step& u = step(ST_TRMM_U);
    StepItem t3;
    t3.dst = dst;
    t3.x = Opnd::slot(z);
    t3.y = Opnd::slot(tmp);
    u.items.push_back(t3);
    pool_.release(tmp);
  }

  // Value of the depth-d node (r, c) in a fresh slot (d may be 0: a plain load).
  int value(int r, int c, int d) {
    if (d == 0) {
      const int out = pool_.alloc();
      Step& ld = step(ST_LOAD);
      StepItem it;
      it.dst = Opnd::slot(out);
      it.x = blk(r, c);
      ld.items.push_back(it);
      return out;
    }
    return eval({Node{r, c, d}}, {-1})[0];
  }

  // Values of a batch of nodes of one depth d >= 1, with the accumulated
  // sums accs subtracted when given.
  std::vector<int> eval_children(const std::vector<Node>& L, const std::vector<int>& accs = {}) {
    if (L.empty()) return {};
    return eval(L, accs.empty() ? std::vector<int>(L.size(), -1) : accs);
  }

  Plan& plan_;
  std::vector<int> elim_;
  const LitTree* lit_ = nullptr;
  int width_;
  SlotPool pool_;
  int node_counter_ = 0;
  int rhs_col_ = -1;
  std::vector<int> memo_;
};

double cube(double x) { return x * x * x; }

void account(Plan& p) {
  const double b = p.b;
  p.launches = 0;
  p.executed_flops = 0;
  for (const Step& s : p.steps) {
    const double n = static_cast<double>(s.items.size());
    switch (s.kind) {
      case ST_LOAD:
        p.launches += 1;
        break;
      case ST_GETRF:
        p.launches += getrf_launches(p.b, lu_kind(static_cast<int>(n), p.b, false, true, 0));
        p.executed_flops += n * getrf_flops(p.b);
        break;
      case ST_TRTRI:
        p.launches += trtri_launches(p.b, lu_kind(static_cast<int>(n), p.b, false, true, 0));
        p.executed_flops += n * trtri_flops(p.b);  // the recursive LU forms the inverses itself
        break;
      case ST_TRMM_L:
      case ST_TRMM_U:
        p.launches += 1;
        p.executed_flops += n * cube(b);
        break;
      default:
        p.launches += 1;
        p.executed_flops += n * 2.0 * cube(b);
        break;
    }
  }
}

}  // namespace

int64_t getrf_launches(int b, LuKind kind) {
  // tile pivoting: two more launches record the element growth
  // recursive: one launch per diagonal tile, four per inner node
  if (kind == LU_RECURSIVE) return 2 + b / kTile + 4 * (b / kTile - 1);
  const bool tile_pivoting = kind == LU_TILE;
  if (tile_pivoting) return 3 + (b > kTile ? (b + kTile - 1) / kTile : 0);  // first tile, one launch per tile
  int64_t n = 0;
  for (int j = 0; j < b;) {
    const int w = std::min(panel_width(b - j), b - j);
    n += 1;                          // panel
    if (j > 0 || j + w < b) n += 1;  // row interchanges (+ triangular solve)
    if (j + w < b) n += 1;           // trailing update
    j += w;
  }
  return n;
}

int64_t trtri_launches(int b, LuKind kind) {
  if (kind == LU_RECURSIVE) return 0;
  int64_t n = kind == LU_TILE ? 0 : 1;  // diagonal tiles (left inverted by the tile-pivoting LU)
  for (int s = kTrtriTile; s < b; s *= 2) n += 2;
  return n;
}

double getrf_flops(int b) { return 2.0 / 3.0 * cube(b); }
double trtri_flops(int b) { return 2.0 / 3.0 * cube(b); }

Plan make_block_plan(int64_t n, int k, int i, int j, int width) {
  if (k < 2 || n < k || i < 0 || i >= k || j < 0 || j >= k) throw std::invalid_argument("bad target");
  Plan plan;
  plan.n = n;
  plan.k = k;
  plan.i = i;
  plan.j = j;
  plan.b = static_cast<int>((n + k - 1) / k);
  const int64_t leaves = static_cast<int64_t>(std::pow(4.0, std::max(0, k - 2)));
  plan.width = std::max<int64_t>(1, std::min<int64_t>(width, leaves));
  // Final 2 x 2 frame [[a, c], ...] and elimination sequence (oracle reading:
  // i == j: a = i, c = largest index != i; i != j: a = j, c = i).
  int a, c;
  if (i == j) {
    a = i;
    c = (i == k - 1) ? k - 2 : k - 1;
  } else {
    a = j;
    c = i;
  }
  std::vector<int> elim;
  for (int t = 0; t < k; ++t)
    if (t != a && t != c) elim.push_back(t);
  elim.push_back(c);
  Builder B(plan, elim, plan.width);
  SlotPool& pool = B.pool();
  const int depth = k - 1;
  int sz = -1;
  int sx = -1;
  if (depth == 1) {
    // k = 2: the root itself reads blocks of M.
    int sp = pool.alloc();
    sx = pool.alloc();
    Step& ld = B.step(ST_LOAD);
    StepItem it;
    it.dst = Opnd::slot(sp);
    it.x = Opnd::mblk(c, c);
    ld.items.push_back(it);
    B.factor_and_solve({sp}, {Opnd::mblk(c, a)}, {Opnd::slot(sx)}, true);
    pool.release(sp);
    sz = pool.alloc();
    Step& g = B.step(ST_GEMM);
    StepItem gi;
    gi.dst = Opnd::slot(sz);
    gi.x = Opnd::mblk(a, c);
    gi.y = Opnd::slot(sx);
    gi.cin = Opnd::mblk(a, a);
    g.items.push_back(gi);
  } else if (plan.width >= 4) {
    // Expand the root: its four children are evaluated as one batch.
    const std::vector<int> r4 = B.eval({Node{a, a, depth - 1}, Node{a, c, depth - 1}, Node{c, c, depth - 1},
                                        Node{c, a, depth - 1}},
                                       {-1, -1, -1, -1});
    sz = r4[0];
    const int sc_ = r4[1], sp = r4[2];
    sx = r4[3];
    B.factor_and_solve({sp}, {Opnd::slot(sx)}, {Opnd::slot(sx)}, true);
    pool.release(sp);
    Step& g = B.step(ST_GEMM);
    StepItem gi;
    gi.dst = Opnd::slot(sz);
    gi.x = Opnd::slot(sc_);
    gi.y = Opnd::slot(sx);
    gi.cin = Opnd::slot(sz);
    g.items.push_back(gi);
    pool.release(sc_);
  } else {
    // Branch by branch (W = 1): pivot child, factor, right child, solve, left
    // child into the running sum, diagonal child.
    const int sp = B.value(c, c, depth - 1);
    B.factor_only({sp});
    sx = B.value(c, a, depth - 1);
    B.solve_only({sp}, {sx});
    pool.release(sp);
    const int sc_ = B.value(a, c, depth - 1);
    const int acc = pool.alloc();
    Step& g = B.step(ST_GEMM_ACC);
    StepItem gi;
    gi.dst = Opnd::slot(acc);
    gi.x = Opnd::slot(sc_);
    gi.y = Opnd::slot(sx);
    g.items.push_back(gi);
    pool.release(sc_);
    if (i == j) {
      pool.release(sx);  // X is only needed for the off-diagonal block
      sx = -1;
    }
    sz = B.eval({Node{a, a, depth - 1}}, {acc})[0];
    pool.release(acc);
  }
  // N_aa = Z^{-1}; for i != j, N_ij = -X N_aa (lower-left block of eq. invSchur).
  if (i == j) {
    B.final_inverse(sz, Opnd::outp(), true);
  } else {
    int sn = pool.alloc();
    B.final_inverse(sz, Opnd::slot(sn), true);
    Step& g = B.step(ST_GEMM_NEG);
    StepItem gi;
    gi.dst = Opnd::outp();
    gi.x = Opnd::slot(sx);
    gi.y = Opnd::slot(sn);
    g.items.push_back(gi);
    pool.release(sn);
  }
  if (sx >= 0) pool.release(sx);
  pool.release(sz);
  plan.nslots = pool.peak;
  const double b3 = cube(plan.b);
  const double T = static_cast<double>((static_cast<int64_t>(std::pow(4.0, k - 1)) - 1) / 3);
  plan.algorithmic_flops = T * (14.0 / 3.0) * b3 + 2.0 * b3 + (i != j ? 2.0 * b3 : 0.0);
  account(plan);
  return plan;
}

Plan make_block_plan_literal(int64_t n, int k, int i, int j, int width) {
  if (k < 2 || n < k || i < 0 || i >= k || j < 0 || j >= k) throw std::invalid_argument("bad target");
  Plan plan;
  plan.n = n;
  plan.k = k;
  plan.i = i;
  plan.j = j;
  plan.b = static_cast<int>((n + k - 1) / k);
  const int64_t leaves = static_cast<int64_t>(std::pow(4.0, std::max(0, k - 2)));
  plan.width = std::max<int64_t>(1, std::min<int64_t>(width, leaves));
  const LitTree tree(k, i, j);
  Builder B(plan, {}, plan.width);
  B.set_literal(&tree);
  // The root frame reduces to the (M/D) of the permuted matrix, whose inverse
  // is the target block (eq. blockmatrix_NxN); every target, diagonal or
  // not, ends with that one inversion.
  const int sz = B.eval({Node{-1, -1, k - 1, tree.root()}}, {-1})[0];
  B.final_inverse(sz, Opnd::outp(), true);
  B.pool().release(sz);
  plan.nslots = B.pool().peak;
  const double b3 = cube(plan.b);
  const double T = static_cast<double>((static_cast<int64_t>(std::pow(4.0, k - 1)) - 1) / 3);
  plan.algorithmic_flops = T * (14.0 / 3.0) * b3 + 2.0 * b3;
  account(plan);
  return plan;
}

namespace {

// Factored elimination pivots P_pos = v(order[pos], order[pos], {order[0..pos-1]})
// for pos < npos, in increasing position: each is evaluated with the pivots
// before it kept (three children per Schur node instead of four) and stays in
// its slot (kept[pos]).  This is the reuse across branches the paper
// suggests as future work (Section "Conclusion").
void build_pivots(Builder& B, const std::vector<int>& order, int npos, std::vector<int>& kept) {
  kept.clear();
  for (int pos = 0; pos < npos; ++pos) {
    B.set_memo(kept);
    const int sq = B.value(order[pos], order[pos], pos);
    B.factor_only({sq});
    B.plan_.schur_ops--;  // a kept pivot's factorisation, counted with the inversions
    B.plan_.final_inversions++;
    kept.push_back(sq);
  }
  B.set_memo(kept);
}

}  // namespace

Plan make_block_plan_reuse(int64_t n, int k, int i, int j, int width) {
  if (k < 2 || n < k || i < 0 || i >= k || j < 0 || j >= k) throw std::invalid_argument("bad target");
  if (k == 2) return make_block_plan(n, k, i, j, width);  // nothing to reuse
  Plan plan;
  plan.n = n;
  plan.k = k;
  plan.i = i;
  plan.j = j;
  plan.b = static_cast<int>((n + k - 1) / k);
  const int64_t leaves = static_cast<int64_t>(std::pow(3.0, std::max(0, k - 2)));
  plan.width = std::max<int64_t>(1, std::min<int64_t>(width, leaves));
  int a, c;
  if (i == j) {
    a = i;
    c = (i == k - 1) ? k - 2 : k - 1;
  } else {
    a = j;
    c = i;
  }
  std::vector<int> elim;
  for (int t = 0; t < k; ++t)
    if (t != a && t != c) elim.push_back(t);
  elim.push_back(c);
  Builder B(plan, elim, plan.width);
  SlotPool& pool = B.pool();
  std::vector<int> kept;
  build_pivots(B, elim, k - 2, kept);
  // Root frame values at depth k - 2 (every pivot below them kept), then the
  // root pivot v(c, c) and the final 2 x 2 step as in the recomputing plan.
  const std::vector<int> r4 = B.eval_children({Node{a, a, k - 2}, Node{a, c, k - 2}, Node{c, c, k - 2},
                                               Node{c, a, k - 2}});
  const int sz = r4[0], sc_ = r4[1], sp = r4[2], sx = r4[3];
  B.factor_and_solve({sp}, {Opnd::slot(sx)}, {Opnd::slot(sx)}, true);
  pool.release(sp);
  {
    Step& g = B.step(ST_GEMM);
    StepItem gi;
    gi.dst = Opnd::slot(sz);
    gi.x = Opnd::slot(sc_);
    gi.y = Opnd::slot(sx);
    gi.cin = Opnd::slot(sz);
    g.items.push_back(gi);
  }
  pool.release(sc_);
  if (i == j) {
    B.final_inverse(sz, Opnd::outp(), true);
  } else {
    int sn = pool.alloc();
    B.final_inverse(sz, Opnd::slot(sn), true);
    Step& g = B.step(ST_GEMM_NEG);
    StepItem gi;
    gi.dst = Opnd::outp();
    gi.x = Opnd::slot(sx);
    gi.y = Opnd::slot(sn);
    g.items.push_back(gi);
    pool.release(sn);
  }
  pool.release(sx);
  pool.release(sz);
  for (int kp : kept) pool.release(kp);
  plan.nslots = pool.peak;
  const double b3 = cube(plan.b);
  const double T = static_cast<double>((static_cast<int64_t>(std::pow(4.0, k - 1)) - 1) / 3);
  plan.algorithmic_flops = T * (14.0 / 3.0) * b3 + 2.0 * b3 + (i != j ? 2.0 * b3 : 0.0);
  account(plan);
  return plan;
}

namespace {

// Elimination order of the block column plans: every index but j ascending,
// j last (x_j is the first unknown of the back substitution).
std::vector<int> column_order(int k, int j) {
  std::vector<int> order;
  for (int t = 0; t < k; ++t)
    if (t != j) order.push_back(t);
  return order;
}

void init_column_plan(Plan& plan, int64_t n, int k, int j, int width) {
  if (k < 2 || n < k || j < 0 || j >= k) throw std::invalid_argument("bad target");
  plan.n = n;
  plan.k = k;
  plan.i = -1;
  plan.j = j;
  plan.b = static_cast<int>((n + k - 1) / k);
  const int64_t leaves = static_cast<int64_t>(std::pow(4.0, std::max(0, k - 2)));
  plan.width = std::max<int64_t>(1, std::min<int64_t>(width, leaves));
}

// Block column j of Gamma^{-1} by block back substitution:
//   x_j = v(j, j, P)^{-1}, P = every other index;
//   x_q = -v(q, q, I_q)^{-1} (v(q, j, I_q) x_j + sum_{t after q} v(q, t, I_q) x_t).
// With kept != nullptr the factored pivot of every position stays in its slot
// (kept[pos], pos = position in the elimination order, j at k - 1).
void build_column(Builder& B, const std::vector<int>& order, int j, std::vector<int>* kept) {
  Plan& plan = B.plan_;
  const int k = plan.k;
  SlotPool& pool = B.pool();
  if (kept) kept->assign(k, -1);
  {
    const int sz = B.value(j, j, k - 1);
    B.final_inverse(sz, Opnd::out_blk(j), true);
    if (kept)
      (*kept)[k - 1] = sz;
    else
      pool.release(sz);
  }
  for (int pos = k - 2; pos >= 0; --pos) {
    const int q = order[pos];
    std::vector<int> later(order.begin() + pos + 1, order.end());
    later.insert(later.begin(), j);
    // All values of this position have depth pos: one lock-step batch
    // (pivot last); at depth 0 they are blocks of Gamma read in place.
    std::vector<Node> nodes;
    for (int t : later) nodes.push_back(Node{q, t, pos});
    nodes.push_back(Node{q, q, pos});
    std::vector<int> sv(nodes.size(), -1);
    if (pos > 0) sv = B.eval_children(nodes);
    int acc = pool.alloc();
    for (size_t u = 0; u < later.size(); ++u) {
      Step& g = B.step(ST_GEMM);
      StepItem it;
      it.dst = Opnd::slot(acc);
      it.x = pos > 0 ? Opnd::slot(sv[u]) : Opnd::mblk(q, later[u]);
      it.y = Opnd::out_blk(later[u]);
      it.cin = u == 0 ? Opnd::none() : Opnd::slot(acc);
      g.items.push_back(it);
      if (pos > 0) pool.release(sv[u]);
    }
    const int sq = pos > 0 ? sv.back() : B.value(q, q, 0);
    B.factor_only({sq});
    plan.schur_ops--;  // the back-substitution pivots are inversions, not Schur steps
    plan.final_inversions++;
    B.solve_only({sq}, {acc});
    Step& cp = B.step(ST_LOAD);
    StepItem it;
    it.dst = Opnd::out_blk(q);
    it.x = Opnd::slot(acc);
    cp.items.push_back(it);
    if (kept)
      (*kept)[pos] = sq;
    else
      pool.release(sq);
    pool.release(acc);
  }
}

}  // namespace

Plan make_column_plan(int64_t n, int k, int j, int width) {
  Plan plan;
  init_column_plan(plan, n, k, j, width);
  const std::vector<int> order = column_order(k, j);
  Builder B(plan, order, plan.width);
  build_column(B, order, j, nullptr);
  plan.nslots = B.pool().peak;
  plan.algorithmic_flops = 0;
  account(plan);
  return plan;
}

// Blocks of Gamma read by the products of a step are first converted into
// slots by a load step (numbered from `base`, live for that step only), so
// that the products of a float recursion only read float slots while M
// stays in its own precision; returns the most slots one step needed.
int stage_matrix_blocks(Plan& p, int base) {
  std::vector<Step> out;
  out.reserve(p.steps.size() * 2);
  int most = 0;
  for (Step& st : p.steps) {
    if (st.kind == ST_LOAD || st.kind == ST_GETRF || st.kind == ST_TRTRI) {
      out.push_back(std::move(st));
      continue;
    }
    std::vector<std::pair<int, int>> blocks;  // unique (r, c) in first-use order
    auto slot_of = [&](Opnd& o) {
      if (o.kind != OPND_MBLK) return;
      const std::pair<int, int> rc(o.a, o.b);
      size_t u = 0;
      while (u < blocks.size() && blocks[u] != rc) ++u;
      if (u == blocks.size()) blocks.push_back(rc);
      o = Opnd::slot(base + static_cast<int>(u));
    };
    for (StepItem& it : st.items) {
      slot_of(it.x);
      slot_of(it.y);
      slot_of(it.cin);
      slot_of(it.sub);
    }
    if (!blocks.empty()) {
      Step ld{ST_LOAD, {}};
      for (size_t u = 0; u < blocks.size(); ++u) {
        StepItem it;
        it.dst = Opnd::slot(base + static_cast<int>(u));
        it.x = Opnd::mblk(blocks[u].first, blocks[u].second);
        ld.items.push_back(it);
      }
      out.push_back(std::move(ld));
      most = std::max(most, static_cast<int>(blocks.size()));
    }
    out.push_back(std::move(st));
  }
  p.steps = std::move(out);
  return most;
}

Plan make_block_plan_staged(int64_t n, int k, int i, int j, int width) {
  Plan p = make_block_plan(n, k, i, j, width);
  p.nslots += stage_matrix_blocks(p, p.nslots);
  account(p);
  return p;
}

RefinePlans make_refine_plans(int64_t n, int k, int j, int width, bool reuse) {
  RefinePlans rp;
  init_column_plan(rp.column, n, k, j, width);
  init_column_plan(rp.solve, n, k, j, width);
  std::vector<int> order = column_order(k, j);
  Builder B(rp.column, order, rp.column.width);
  if (reuse) {
    // Only the pivots: every position's pivot with the earlier ones kept;
    // the block column itself then comes from the solve plan with R = E_j.
    std::vector<int> full(order);
    full.push_back(j);
    build_pivots(B, full, k, rp.kept);
    rp.column_gives_x0 = false;
  } else {
    build_column(B, order, j, &rp.kept);
    rp.column_gives_x0 = true;
  }
  // The solve plan starts from the column plan's pool: the kept pivots stay
  // allocated, everything else is free again.
  Builder S(rp.solve, order, rp.solve.width);
  S.pool() = B.pool();
  S.set_rhs_column(k);
  S.set_memo(std::vector<int>(rp.kept.begin(), rp.kept.end() - 1));
  SlotPool& pool = S.pool();
  // Forward elimination of R rides along as the extra column k; back
  // substitution with the kept pivots:
  //   x_j = v(j, j, P)^{-1} v(j, R, P),
  //   x_q = v(q, q, I_q)^{-1} (v(q, R, I_q) - sum_{t after q} v(q, t, I_q) x_t).
  order.push_back(j);
  for (int pos = k - 1; pos >= 0; --pos) {
    const int q = order[pos];
    // Every value of this position in one lock-step batch (the right-hand
    // side first); at depth 0 they are read in place.
    std::vector<Node> nodes{Node{q, k, pos}};
    for (int t = pos + 1; t < k; ++t) nodes.push_back(Node{q, order[t], pos});
    std::vector<int> sv(nodes.size(), -1);
    if (pos > 0) sv = S.eval_children(nodes);
    const int acc = pos > 0 ? sv[0] : S.value(q, k, 0);
    for (int t = pos + 1; t < k; ++t) {
      Step& g = S.step(ST_GEMM);
      StepItem it;
      it.dst = Opnd::slot(acc);
      it.x = pos > 0 ? Opnd::slot(sv[t - pos]) : Opnd::mblk(q, order[t]);
      it.y = Opnd::out_blk(order[t]);
      it.cin = Opnd::slot(acc);
      g.items.push_back(it);
      if (pos > 0) pool.release(sv[t - pos]);
    }
    S.solve_with({rp.kept[pos]}, {Opnd::slot(acc)}, {Opnd::out_blk(q)});
    pool.release(acc);
  }
  rp.column.nslots = rp.solve.nslots = std::max(B.pool().peak, pool.peak);
  // The float recursion reads M only through staged loads (converted to
  // float, scaled, identity padding synthesised) into slots past the plans'.
  const int base = rp.column.nslots;
  const int staged = std::max(stage_matrix_blocks(rp.column, base), stage_matrix_blocks(rp.solve, base));
  rp.column.nslots = rp.solve.nslots = base + staged;
  rp.column.algorithmic_flops = rp.solve.algorithmic_flops = 0;
  account(rp.column);
  account(rp.solve);
  return rp;
}

}  // namespace bri
